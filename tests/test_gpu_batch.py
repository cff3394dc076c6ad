"""Parity of the batched path (many independent tall-skinny matrices of mixed
heights in one launch) with the CPU oracle, through the C ABI.

Every instance is compared with the oracle's R on the same input (FP64:
relative Frobenius error 1e-10; FP32: 1e-5 against the oracle on the
FP32-rounded input promoted to FP64).  The forward error of R grows with the
condition number of the columns that determine Q (all n when m >= n, the
leading m when m < n), so for FP32 the bound is 1e-5 up to condition number
10 and grows in proportion beyond it: a short, nearly square instance of
uniform entries can have a condition number in the thousands.

A batched instance is also checked bit for bit against the single-matrix
entry point run with the same leaf size: both take the same steps in the same
order, so they must agree exactly.
"""
import numpy as np
import pytest

import oracle
from gates import GRAM32, GRAM64
from paper_1002_4250_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1002_4250_amd import tsqr  # noqa: E402

TOL64 = 1e-10
TOL32 = 1e-5


def relF(X, Y):
    return float(np.linalg.norm(X - Y) / max(np.linalg.norm(Y), 1e-300))


def batch_gpu(flat, sizes, offsets, n, leaf_rows=0):
    h = tsqr.handle(0)
    tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_LEAF_ROWS, leaf_rows)
    try:
        dt = torch.float64 if flat.dtype == np.float64 else torch.float32
        plan = tsqr.BatchPlan(sizes, offsets, n, dt, h=h)
    finally:
        tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_LEAF_ROWS, 0)
    Ad = torch.from_numpy(flat).cuda()
    R = plan.run(Ad)
    torch.cuda.synchronize()
    return R.cpu().numpy(), plan


def tol32(A):
    m, n = A.shape
    k = min(m, n)
    if k == 0:
        return TOL32
    s = np.linalg.svd(A[:, :k], compute_uv=False)
    cond = float(s[0] / s[-1]) if s[-1] > 0 else np.inf
    return TOL32 * max(1.0, cond / 10.0)


def r_of(Rb, b, n):
    # batch entry b holds R column-major: element (i, j) at [b, j, i]
    return Rb[b].T[:n, :n]


def ragged(sizes, n, seed, dtype):
    sizes = np.asarray(sizes, dtype=np.int64)
    offsets = np.zeros(len(sizes), dtype=np.int64)
    if len(sizes) > 1:
        np.cumsum(sizes[:-1] * n, out=offsets[1:])
    flat = np.empty(int(sizes.sum()) * n, dtype=dtype)
    for b, m in enumerate(sizes):
        o = int(offsets[b])
        flat[o:o + int(m) * n] = inputs.batched_instance(b, int(m), n, seed, dtype).T.ravel()
    return flat, sizes, offsets


@pytest.mark.parametrize("n", [1, 7, 16, 17, 50, 64])
@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_ragged_batch_matches_oracle(n, dt):
    sizes = list(inputs.batched_sizes(40, 1, 20000, seed=5)) + [0, 1, 2, n, n + 1, 4096, 4097, 8192]
    flat, sizes, offsets = ragged(sizes, n, 11, dt)
    Rb, plan = batch_gpu(flat, sizes, offsets, n)
    tiles, leaves, L = plan.info()
    assert tiles == leaves == sum(max(1, -(-int(m) // L)) for m in sizes)
    for b, m in enumerate(sizes):
        A = inputs.instance(flat, sizes, offsets, b, n).astype(np.float64)
        Rg = r_of(Rb, b, n)
        if m == 0:
            assert np.all(Rg == 0), b
            continue
        Ro = oracle.r_factor(np.asfortranarray(A))
        tol = TOL64 if dt == np.float64 else tol32(A)
        assert relF(Rg, Ro) < tol, (b, m, tol)
        gate = GRAM64 if dt == np.float64 else GRAM32
        assert oracle.gram_residual(A, Rg.astype(np.float64)) < gate, (b, m)
        assert np.all(np.tril(Rg, -1) == 0) and not np.any(np.signbit(np.diag(Rg))), (b, m)


@pytest.mark.parametrize("dt", [np.float64, np.float32])
def test_batched_instance_equals_single_call_bitwise(dt):
    n = 50
    sizes = [100, 3000, 40000, 1, 70000]
    flat, sizes, offsets = ragged(sizes, n, 3, dt)
    Rb, plan = batch_gpu(flat, sizes, offsets, n)
    _, _, L = plan.info()
    h = tsqr.handle(0)
    tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_LEAF_ROWS, L)
    try:
        for b in range(len(sizes)):
            A = inputs.instance(flat, sizes, offsets, b, n)
            Ad = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
            Rs = tsqr.geqr_r(Ad).cpu().numpy()
            assert np.array_equal(Rs, r_of(Rb, b, n)), b
    finally:
        tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_LEAF_ROWS, 0)


@pytest.mark.parametrize("leaf_rows", [128, 1000, 65536])
def test_batch_leaf_sizes(leaf_rows):
    n = 32
    sizes = list(inputs.batched_sizes(24, 64, 30000, seed=9))
    flat, sizes, offsets = ragged(sizes, n, 4, np.float64)
    Rb, plan = batch_gpu(flat, sizes, offsets, n, leaf_rows=leaf_rows)
    for b in range(len(sizes)):
        A = np.asfortranarray(inputs.instance(flat, sizes, offsets, b, n))
        assert relF(r_of(Rb, b, n), oracle.r_factor(A)) < TOL64, b


def test_batch_reexecution_and_strided_output():
    """Re-running a plan reuses its workspace (tree counters are cleared by
    each run); R may be written with a leading dimension above n."""
    n = 16
    flat, sizes, offsets = ragged([5000, 64, 20000, 333], n, 8, np.float64)
    plan = tsqr.BatchPlan(sizes, offsets, n, torch.float64)
    Ad = torch.from_numpy(flat).cuda()
    first = plan.run(Ad).cpu().numpy()
    for _ in range(3):
        again = plan.run(Ad).cpu().numpy()
        assert np.array_equal(first, again)
    ldr = 19
    Rbuf = torch.full((len(sizes) * n * ldr,), 5.0, dtype=torch.float64, device="cuda")
    st = tsqr.tsqr_batch_exec(plan.plan, Ad.data_ptr(), Rbuf.data_ptr(), ldr, plan.ws.data_ptr(),
                              plan.ws.numel(), tsqr._stream_ptr(torch, Ad.device))
    assert st == 0
    torch.cuda.synchronize()
    buf = Rbuf.cpu().numpy().reshape(len(sizes), n, ldr)
    for b in range(len(sizes)):
        assert np.array_equal(buf[b][:, :n].T, r_of(first, b, n)), b
        assert np.all(buf[b][:, n:] == 5.0)


def test_batch_in_hip_graph_matches_eager():
    """Plan execution holds two kernels and no memset, so it can be captured;
    every replay (with eager work between them) equals the eager result."""
    n = 50
    flat, sizes, offsets = ragged(list(inputs.batched_sizes(64, 64, 65536, seed=3)), n, 6, np.float32)
    plan = tsqr.BatchPlan(sizes, offsets, n, torch.float32)
    Ad = torch.from_numpy(flat).cuda()
    eager = plan.run(Ad).clone()
    R = torch.empty_like(eager)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run(Ad, R)              # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run(Ad, R)
    for i in range(4):
        R.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(R, eager), i
        plan.run(Ad)                 # eager work between replays
        torch.cuda.synchronize()


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_stamped_exec_measures_the_schedule(dt):
    """The stamped exec gives R bit for bit as the plain exec, and a start and
    end on the device clock for every workgroup: ends after starts, the span
    close to the launch's own elapsed time, and no more workgroups at once
    than the device holds."""
    n = 50
    flat, sizes, offsets = ragged(inputs.batched_sizes(300, lo=64, hi=40000, seed=9), n, 9, dt)
    tdt = torch.float64 if dt == np.float64 else torch.float32
    plan = tsqr.BatchPlan(sizes, offsets, n, tdt)
    Ad = torch.from_numpy(flat).cuda()
    R0 = plan.run(Ad).clone()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    R1, stamps = plan.run_stamped(Ad)
    e1.record()
    torch.cuda.synchronize()
    assert torch.equal(R0, R1)
    khz = tsqr.device_clock_khz(tsqr.handle(0))
    st = stamps.cpu().numpy()
    tiles = plan.info()[0]
    assert st.shape == (tiles, 2)
    assert np.all(st[:, 0] > 0) and np.all(st[:, 1] >= st[:, 0])
    span_ms = (st[:, 1].max() - st[:, 0].min()) / khz
    ev_ms = e0.elapsed_time(e1)
    print(f"tiles {tiles}, clock {khz} kHz, span {span_ms:.3f} ms, events {ev_ms:.3f} ms", flush=True)
    assert 0.5 * ev_ms < span_ms <= ev_ms * 1.05 + 0.05
    # concurrency: +1 at each start, -1 at each end (ends first on ties)
    t = np.concatenate([st[:, 0], st[:, 1]])
    d = np.concatenate([np.ones(tiles, np.int64), -np.ones(tiles, np.int64)])
    order = np.lexsort((d, t))
    active = np.cumsum(d[order])
    assert active.min() >= 0 and 1 <= active.max() <= 256 * 8
