"""The shipped tuning table on the GPU: a handle that follows it gives R
within the FP64 / FP32 gates of the oracle, and bit for bit what the plain
handle gives when the same configuration is set by hand (the table only
chooses the launch geometry)."""
import numpy as np
import pytest

import oracle
from paper_1002_4250_amd import autotune, inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1002_4250_amd import tsqr  # noqa: E402

TABLE = autotune.load()
if TABLE is None:
    pytest.skip("no tuning table shipped", allow_module_level=True)


@pytest.fixture(scope="module")
def tuned():
    h = tsqr.tsqr_create(0)
    assert autotune.apply(h, TABLE) == len(TABLE["entries"])
    yield h
    tsqr.tsqr_destroy(h)


def relF(X, Y):
    return float(np.linalg.norm(X - Y) / np.linalg.norm(Y))


def entry_for(dtype, m):
    cands = [e for e in TABLE["entries"] if e["dtype"] == dtype and not e["batch"] and m <= e["m_max"]]
    return min(cands, key=lambda e: e["m_max"])


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("m", [3000, 20000, 70000, 300000])
def test_tuned_plain_matches_oracle_and_manual_config(tuned, dtype, m):
    n = 50
    A = inputs.uniform(m, n, 7)
    if dtype == "f32":
        A = A.astype(np.float32)
    Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
    Rt = tsqr.geqr_r(Ad, h=tuned).cpu().numpy()
    Ro = oracle.r_factor(np.asfortranarray(A.astype(np.float64)))
    assert relF(Rt, Ro) < (1e-10 if dtype == "f64" else 1e-5)
    # the same configuration set by hand on a handle without a table
    e = entry_for(dtype, m)
    code = autotune.DTYPES[dtype]
    h = tsqr.tsqr_create(0)
    try:
        tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_ROWS_PER_LANE, e["rows_per_lane"])
        tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_WAVES_PER_CU, e["waves_per_cu"])
        assert tsqr.tsqr_plan_info(h, m, n, code) == tsqr.tsqr_plan_info(tuned, m, n, code)
        Rm = tsqr.geqr_r(Ad, h=h).cpu().numpy()
    finally:
        tsqr.tsqr_destroy(h)
    assert np.array_equal(Rt, Rm)


def test_tuned_batch_matches_oracle(tuned):
    n = 50
    flat, sizes, offsets = inputs.batched_uniform(256, n, 64, 65536, seed=4, dtype=np.float32)
    plan = tsqr.BatchPlan(sizes, offsets, n, torch.float32, h=tuned)
    e = [x for x in TABLE["entries"] if x["dtype"] == "f32" and x["batch"]][0]
    assert plan.info()[2] == e["leaf_rows"]
    Rb = plan.run(torch.from_numpy(flat).cuda()).cpu().numpy()
    for b in (0, 17, int(np.argmax(sizes)), int(np.argmin(sizes)), 255):
        A = np.asfortranarray(inputs.instance(flat, sizes, offsets, b, n).astype(np.float64))
        s = np.linalg.svd(A, compute_uv=False)
        tol = 1e-5 * max(1.0, float(s[0] / s[-1]) / 10.0)
        assert relF(Rb[b].T, oracle.r_factor(A)) < tol, b


def test_tuner_runs_end_to_end():
    """A small tuning run (one bucket, one element type, a small batch)
    produces a table whose entries are the fastest of their candidates and
    that a fresh handle accepts."""
    table = autotune.tune(n=16, dtypes=("f32",), buckets=[4096], batch_count=64, reps=2)
    ents = table["entries"]
    assert [e["batch"] for e in ents] == [False, True]
    for e in ents:
        assert e["us"] == min(c[2] for c in e["candidates"]) > 0
    h = tsqr.tsqr_create(0)
    try:
        assert autotune.apply(h, table) == 2
    finally:
        tsqr.tsqr_destroy(h)
