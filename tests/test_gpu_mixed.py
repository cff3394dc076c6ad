"""Mixed precision (FP32 TSQR followed by one FP64 Cholesky-based correction)
against the CPU oracle, through the C ABI.

The oracle is the definition (FP64 Householder QR) run on the FP32-stored
input promoted to FP64.  Every instance must meet three gates (tests/gates.py):
the global forward error relF <= 1e-13 * max(1, kappa); the backward error
||R^T R - A^T A||_F / ||A||_F^2 <= 1e-14, independent of kappa; and the
row-scaled forward error <= 1e-14 * max(1, kappa)^0.6, which sees the small
trailing rows.  The last two are what an FP32-accurate R cannot meet: a
control checks that the uncorrected FP32 factor fails them from kappa = 1e6
up (it passes the relF gate there).  Instances whose Gram matrix is not
numerically positive definite must be reported as refactored in FP64 and meet
the same gates.
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


def run_mixed(flat, batch, m, n):
    plan = tsqr.MixedPlan(batch, m, n)
    R, fb = plan.run(torch.from_numpy(flat).cuda())
    torch.cuda.synchronize()
    return R.cpu().numpy(), fb, plan


@pytest.mark.parametrize("m,n", [(4096, 50), (3000, 17), (700, 64), (9000, 32)])
def test_mixed_matches_oracle_over_kappa(m, n):
    batch = 9
    flat, kappas = inputs.conditioned_batch(batch, m, n, log10_kappa_max=8.0, seed=7)
    Rb, fb, _ = run_mixed(flat, batch, m, n)
    for b in range(batch):
        A = np.asfortranarray(flat[b * m * n:(b + 1) * m * n].reshape(n, m).T.astype(np.float64))
        Ro = oracle.r_factor(A)
        Rg = Rb[b].T
        tol = 1e-13 * max(1.0, kappas[b])
        assert relF(Rg, Ro) < tol, (b, kappas[b], fb[b], relF(Rg, Ro))
        assert oracle.gram_residual(A, Rg) < GRAM64, (b, kappas[b], oracle.gram_residual(A, Rg))
        k = kappa_of(Ro)
        assert row_scaled(Rg, Ro) < row_gate64(k), (b, k, row_scaled(Rg, Ro))
        assert np.all(np.tril(Rg, -1) == 0) and np.all(np.diag(Rg) > 0), b
    # well-conditioned instances take the corrected FP32 path
    assert all(fb[b] == 0 for b in range(batch) if kappas[b] <= 1e4), fb


def test_mixed_falls_back_when_cholesky_fails():
    """An exactly rank-deficient instance (a zero column: its reflector is the
    identity, so R~ has an exact zero on the diagonal) gives a singular R~,
    so its Gram matrix cannot be factored: the instance is reported and
    refactored by the plain FP64 path from its FP32 storage (a batched launch
    with leaves of 64 chunks, decided on the device), whose result it must
    equal bit for bit: the single-matrix FP64 call on the promoted values with
    the same leaf size takes the same steps.  R is not unique past the zero
    pivot, so against the data only the Gram identity is checked."""
    m, n = 2048, 50
    A = inputs.conditioned(m, n, 10.0, seed=11)
    A[:, 7] = 0.0
    B = inputs.conditioned(m, n, 10.0, seed=12)
    flat = np.concatenate([A.T.ravel(), B.T.ravel()])
    Rb, fb, _ = run_mixed(flat, 2, m, n)
    assert fb == [1, 0]
    A64 = A.astype(np.float64)
    h = tsqr.handle(0)
    tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_LEAF_ROWS, 64 * 128)
    try:
        Rs = tsqr.geqr_r(torch.from_numpy(np.ascontiguousarray(A64.T)).cuda().t(), h=h).cpu().numpy()
    finally:
        tsqr.tsqr_set_option(h, tsqr.TSQR_OPT_LEAF_ROWS, 0)
    assert np.array_equal(Rb[0].T, Rs)
    G = A64.T @ A64
    assert np.linalg.norm(Rs.T @ Rs - G) / np.linalg.norm(G) < 1e-13
    Ro = oracle.r_factor(np.asfortranarray(B.astype(np.float64)))
    assert relF(Rb[1].T, Ro) < 1e-12


def test_mixed_is_more_accurate_than_fp32():
    """The correction is what brings FP32 storage to FP64 accuracy."""
    m, n = 8192, 50
    A = inputs.conditioned(m, n, 1e3, seed=12)
    flat = A.T.ravel().copy()
    Rb, fb, _ = run_mixed(flat, 1, m, n)
    assert fb == [0]
    Ro = oracle.r_factor(np.asfortranarray(A.astype(np.float64)))
    R32 = tsqr.geqr_r(torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()).cpu().numpy().astype(np.float64)
    e_mixed, e_32 = relF(Rb[0].T, Ro), relF(R32, Ro)
    assert e_mixed < 1e-12 and e_32 > 1e-9, (e_mixed, e_32)


@pytest.mark.parametrize("kappa", [1e6, 1e7, 1e8])
def test_gates_reject_the_uncorrected_fp32_factor(kappa):
    """Control: the FP32 TSQR factor alone fails the backward-error and
    row-scaled gates, which the corrected result meets; from kappa = 1e7 up it
    passes the global relF gate (its error is dominated by the leading rows),
    which is why that gate alone cannot tell the two apart."""
    m, n = 16384, 50
    A = inputs.conditioned(m, n, kappa, seed=31)
    Rb, fb, _ = run_mixed(A.T.ravel().copy(), 1, m, n)
    A64 = np.asfortranarray(A.astype(np.float64))
    Ro = oracle.r_factor(A64)
    k = kappa_of(Ro)
    R32 = tsqr.geqr_r(torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()).cpu().numpy().astype(np.float64)
    if kappa >= 1e7:
        assert relF(R32, Ro) < 1e-13 * max(1.0, kappa)             # relF alone is blind here
    assert oracle.gram_residual(A64, R32) > GRAM64 * 100, oracle.gram_residual(A64, R32)
    assert row_scaled(R32, Ro) > row_gate64(k) * 10, (row_scaled(R32, Ro), row_gate64(k))
    Rg = Rb[0].T
    assert oracle.gram_residual(A64, Rg) < GRAM64 and row_scaled(Rg, Ro) < row_gate64(k), fb


def test_mixed_bitwise_reproducible_and_strided():
    m, n, batch = 5000, 50, 3
    flat, _ = inputs.conditioned_batch(batch, m, n, log10_kappa_max=4.0, seed=13)
    R1, fb1, plan = run_mixed(flat, batch, m, n)
    Ad = torch.from_numpy(flat).cuda()
    R2, fb2 = plan.run(Ad)
    assert fb1 == fb2 and np.array_equal(R1, R2.cpu().numpy())
    # the same instances with a leading dimension above m and a larger stride
    lda, stride = m + 3, (m + 3) * n + 10
    big = np.full(batch * stride, np.nan, dtype=np.float32)
    for b in range(batch):
        inst = flat[b * m * n:(b + 1) * m * n].reshape(n, m)
        for j in range(n):
            big[b * stride + j * lda: b * stride + j * lda + m] = inst[j]
    p2 = tsqr.MixedPlan(batch, m, n, stride=stride, lda=lda)
    R3, fb3 = p2.run(torch.from_numpy(big).cuda())
    torch.cuda.synchronize()
    assert fb3 == fb1
    R3 = R3.cpu().numpy()
    for b in range(batch):
        A = np.asfortranarray(flat[b * m * n:(b + 1) * m * n].reshape(n, m).T.astype(np.float64))
        assert relF(R3[b].T, oracle.r_factor(A)) < 1e-9, b


def test_mixed_in_hip_graph_matches_eager():
    """The call is asynchronous (kernel launches only; the fallback decision is
    taken on the device), so it can be captured in a HIP graph: every replay,
    with eager work between them, equals the eager result, including an
    exactly rank-deficient instance (a zero column) that takes the FP64
    fallback inside the graph."""
    m, n, batch = 4096, 50, 5
    flat, _ = inputs.conditioned_batch(batch, m, n, log10_kappa_max=8.0, seed=17)
    B = inputs.conditioned(m, n, 10.0, seed=18)
    B[:, 9] = 0.0                                  # instance 2: a zero column
    flat[2 * m * n:3 * m * n] = B.T.ravel()
    plan = tsqr.MixedPlan(batch, m, n)
    Ad = torch.from_numpy(flat).cuda()
    eager_R, eager_fb = plan.run(Ad)
    torch.cuda.synchronize()
    assert eager_fb == [0, 0, 1, 0, 0]
    R = torch.empty_like(eager_R)
    flags = torch.zeros(batch, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.launch(Ad, R, flags)                  # warm up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.launch(Ad, R, flags)
    for i in range(4):
        R.fill_(float("nan"))
        flags.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(R, eager_R), i
        assert flags.cpu().tolist() == eager_fb, i
        plan.run(Ad)                               # eager work between replays
        torch.cuda.synchronize()
