"""The sampled preconditioner (R~ from the FP32 TSQR of a stratified row
sample, then the FP64 correction over all of A) against the CPU oracle,
through the C ABI.

The result must be the R of A whatever rows were sampled, so every instance
meets the same three gates as the plain mixed path (tests/gates.py): relF <=
1e-13 max(1, kappa), the backward error ||R^T R - A^T A||_F / ||A||_F^2 <=
1e-14, and the row-scaled forward error <= 1e-14 max(1, kappa)^0.6.  The
sample itself is checked only through what it is for: kappa(A R~^-1) must be
small on the conditioned inputs, and a sample that misses what matters (an
exactly rank-deficient one, or one that misses a dominant row) must send the
instance to the FP64 path rather than give a wrong R.
"""
import numpy as np
import pytest

import oracle
from gates import GRAM64, kappa_of, row_gate64, row_scaled
from paper_1002_4250_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_1002_4250_amd import tsqr  # noqa: E402


def relF(X, Y):
    return float(np.linalg.norm(X - Y) / max(np.linalg.norm(Y), 1e-300))


def instance(flat, b, m, n):
    return np.asfortranarray(flat[b * m * n:(b + 1) * m * n].reshape(n, m).T.astype(np.float64))


def check_gates(A, Rg, kappa, what):
    """kappa: the generator's condition number, or None to take it from the
    oracle's R."""
    Ro = oracle.r_factor(A)
    if kappa is None:
        kappa = kappa_of(Ro)
    assert relF(Rg, Ro) < 1e-13 * max(1.0, kappa), (what, relF(Rg, Ro))
    assert oracle.gram_residual(A, Rg) < GRAM64, (what, oracle.gram_residual(A, Rg))
    k = kappa_of(Ro)
    assert row_scaled(Rg, Ro) < row_gate64(k), (what, k, row_scaled(Rg, Ro))
    assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) > 0), what
    return Ro


@pytest.mark.parametrize("m,n,s,batch", [(65536, 50, 4096, 4), (9000, 32, 1024, 5), (3000, 17, 160, 5),
                                         (700, 64, 320, 3)])
def test_sampled_matches_oracle_over_kappa(m, n, s, batch):
    flat, kappas = inputs.conditioned_batch(batch, m, n, log10_kappa_max=8.0, seed=41)
    plan = tsqr.MixedPlan(batch, m, n, sample_rows=s, seed=5)
    R, fb = plan.run(torch.from_numpy(flat).cuda())
    torch.cuda.synchronize()
    R, Rt = R.cpu().numpy(), plan.rtilde().cpu().numpy().astype(np.float64)
    for b in range(batch):
        A = instance(flat, b, m, n)
        Ro = check_gates(A, R[b].T, kappas[b], (b, kappas[b], fb[b]))
        # A R~^-1 = Q (Ro R~^-1): the sample is a good preconditioner here,
        # up to the FP32 rounding of R~ (about kappa 2^-24, as for the plain
        # mixed path)
        ky = np.linalg.cond(Ro @ np.linalg.inv(np.triu(Rt[b].T)))
        assert ky < 3.0 * (1.0 + kappas[b] * 2.0 ** -24), (b, kappas[b], ky)
    assert fb == [0] * batch, fb


def test_sampled_coherent_row_stays_correct():
    """One row 1e6 times larger than the others: a sample that misses it gives
    an R~ under which A R~^-1 is badly conditioned, and the bound on
    kappa(A R~^-1) must then send the instance to the FP64 path; a sample that
    holds it is a good preconditioner.  Either way R is that of A."""
    m, n = 8192, 50
    outs = []
    for seed in (1, 2, 3):
        A = inputs.conditioned(m, n, 10.0, seed=60 + seed).astype(np.float64)
        A[1234, :] *= 1e6
        A32 = A.astype(np.float32)
        plan = tsqr.MixedPlan(1, m, n, sample_rows=512, seed=seed)
        R, fb = plan.run(torch.from_numpy(A32.T.ravel().copy()).cuda())
        torch.cuda.synchronize()
        check_gates(np.asfortranarray(A32.astype(np.float64)), R[0].cpu().numpy().T, None, (seed, fb))
        outs.append(fb[0])
    # 512 of 8192 rows: most samples miss the row and must have fallen back
    assert sum(outs) >= 1, outs


def test_sampled_zero_column_falls_back():
    """A zero column is zero in every sample, so R~ is exactly singular: the
    instance is reported and refactored by the FP64 path (bit for bit the
    single-matrix FP64 call with the fallback's leaf size); the other instance
    is corrected."""
    m, n = 4096, 50
    A = inputs.conditioned(m, n, 10.0, seed=71)
    A[:, 3] = 0.0
    B = inputs.conditioned(m, n, 1e6, seed=72)
    flat = np.concatenate([A.T.ravel(), B.T.ravel()])
    plan = tsqr.MixedPlan(2, m, n, sample_rows=512, seed=9)
    Rb, fb = plan.run(torch.from_numpy(flat).cuda())
    torch.cuda.synchronize()
    Rb = Rb.cpu().numpy()
    assert fb == [1, 0]
    h = tsqr.handle(0)
    tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_LEAF_ROWS, 64 * 128)
    try:
        A64 = A.astype(np.float64)
        Rs = tsqr.geqr_r(torch.from_numpy(np.ascontiguousarray(A64.T)).cuda().t(), h=h).cpu().numpy()
    finally:
        tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_LEAF_ROWS, 0)
    assert np.array_equal(Rb[0].T, Rs)
    check_gates(np.asfortranarray(B.astype(np.float64)), Rb[1].T, 1e6, "corrected")


def test_sampled_is_deterministic_and_seeded():
    m, n, batch = 20000, 50, 3
    flat, kappas = inputs.conditioned_batch(batch, m, n, log10_kappa_max=6.0, seed=81)
    Ad = torch.from_numpy(flat).cuda()
    p1 = tsqr.MixedPlan(batch, m, n, sample_rows=1000, seed=11)
    R1, fb1 = p1.run(Ad)
    torch.cuda.synchronize()
    Rt1 = p1.rtilde().clone()
    R2, fb2 = p1.run(Ad)
    torch.cuda.synchronize()
    assert fb1 == fb2 and torch.equal(R1, R2) and torch.equal(Rt1, p1.rtilde())
    p3 = tsqr.MixedPlan(batch, m, n, sample_rows=1000, seed=12)
    R3, fb3 = p3.run(Ad)
    torch.cuda.synchronize()
    assert not torch.equal(Rt1, p3.rtilde())          # another sample
    R3 = R3.cpu().numpy()
    for b in range(batch):
        check_gates(instance(flat, b, m, n), R3[b].T, kappas[b], b)


def test_sample_of_all_rows_is_the_plain_plan():
    m, n, batch = 3000, 50, 2
    flat, _ = inputs.conditioned_batch(batch, m, n, log10_kappa_max=4.0, seed=91)
    Ad = torch.from_numpy(flat).cuda()
    Rp, fbp = tsqr.MixedPlan(batch, m, n).run(Ad)
    Rs, fbs = tsqr.MixedPlan(batch, m, n, sample_rows=2945, seed=3).run(Ad)   # rounds up to 3008 >= m
    torch.cuda.synchronize()
    assert fbp == fbs and torch.equal(Rp, Rs)


def test_sampled_in_hip_graph_matches_eager():
    m, n, batch = 8192, 50, 4
    flat, _ = inputs.conditioned_batch(batch, m, n, log10_kappa_max=8.0, seed=95)
    plan = tsqr.MixedPlan(batch, m, n, sample_rows=512, seed=4)
    Ad = torch.from_numpy(flat).cuda()
    eager_R, eager_fb = plan.run(Ad)
    torch.cuda.synchronize()
    R = torch.empty_like(eager_R)
    flags = torch.zeros(batch, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.launch(Ad, R, flags)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch(Ad, R, flags)
    for i in range(3):
        R.fill_(float("nan"))
        flags.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(R, eager_R), i
        assert flags.cpu().tolist() == eager_fb, i
        plan.run(Ad)
        torch.cuda.synchronize()
