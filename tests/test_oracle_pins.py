"""Pins for the CPU oracle, independent of the oracle itself.

Each test checks the oracle against something the paper or the mathematics
fixes: hand-derived examples, a high-precision brute force, closed forms,
matrices whose exact R is known by construction, LAPACK (the special case of a
single block), and the properties the paper states for the reduction operator
(section 2: binary, essentially associative and commutative, any tree gives
the same R).  A plausible slip in the oracle -- a dropped term, a wrong sign or
index, a transposed operand -- fails at least one of them.
"""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import brute
from paper_1002_4250_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def relF(X, Y):
    return np.linalg.norm(X - Y) / max(np.linalg.norm(Y), 1e-300)


def sign_fix(R):
    """Rows scaled so that the diagonal is non-negative (numpy, not the oracle)."""
    s = np.where(np.signbit(np.diag(R)), -1.0, 1.0)
    return R * s[:, None]


def read_hand_examples():
    cases = []
    with open(os.path.join(GOLDEN, "hand_examples.txt")) as f:
        lines = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    i = 0
    while i < len(lines):
        _, name, m, n = lines[i]
        m, n = int(m), int(n)
        A = np.array([[float(v) for v in lines[i + 1 + r]] for r in range(m)])
        R = np.array([[float(v) for v in lines[i + 1 + m + r]] for r in range(n)])
        cases.append((name, A, R))
        i += 1 + m + n
    return cases


def read_brute_small():
    cases = []
    with open(os.path.join(GOLDEN, "brute_small.txt")) as f:
        lines = [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]
    i = 0
    while i < len(lines):
        _, m, n, seed = lines[i]
        m, n = int(m), int(n)
        A = np.array([[float.fromhex(v) for v in lines[i + 1 + j][1:]] for j in range(n)]).T
        R = np.zeros((n, n))
        for r in range(n):
            R[r, r:] = [float.fromhex(v) for v in lines[i + 1 + n + r][1:]]
        cases.append((m, n, int(seed), A, R))
        i += 1 + 2 * n
    return cases


# ---------------------------------------------------------------- definition O1

@pytest.mark.parametrize("case", read_hand_examples(), ids=lambda c: c[0])
def test_hand_examples(case):
    _, A, R = case
    np.testing.assert_allclose(oracle.r_factor(A), R, rtol=0, atol=1e-14 * max(1.0, abs(R).max()))
    np.testing.assert_allclose(oracle.tsqr_r(A, 1), R, rtol=0, atol=1e-14 * max(1.0, abs(R).max()))


@pytest.mark.parametrize("case", read_brute_small(), ids=lambda c: f"{c[0]}x{c[1]}")
def test_stored_brute_force(case):
    m, n, seed, A, R = case
    # the stored A is the generator's output: the fixture also pins inputs.uniform
    assert np.array_equal(A, inputs.uniform(m, n, seed))
    assert relF(oracle.r_factor(A), R) < 1e-14


@pytest.mark.parametrize("m,n,seed", [(1, 1, 0), (3, 3, 1), (7, 2, 2), (12, 5, 3), (40, 7, 4), (5, 5, 5)])
def test_brute_force(m, n, seed):
    A = inputs.uniform(m, n, seed)
    Rb = brute.r_factor(A)
    assert relF(oracle.r_factor(A), Rb) < 1e-14
    for leaf in (1, 2, 3, 8):
        assert relF(oracle.tsqr_r(A, leaf, "binary"), Rb) < 1e-14


def test_n1_closed_form():
    a = inputs.uniform(1000, 1, 7)
    exact = math.sqrt(math.fsum(float(v) * float(v) for v in a[:, 0]))
    assert oracle.r_factor(a)[0, 0] == pytest.approx(exact, rel=1e-15)
    assert oracle.tsqr_r(a, 37)[0, 0] == pytest.approx(exact, rel=1e-14)


def test_n2_closed_form():
    A = inputs.uniform(500, 2, 8)
    a1, a2 = A[:, 0], A[:, 1]
    r11 = math.sqrt(math.fsum(a1 * a1))
    r12 = math.fsum(a1 * a2) / r11
    resid = a2 - (r12 / r11) * a1
    r22 = math.sqrt(math.fsum(resid * resid))
    R = oracle.r_factor(A)
    np.testing.assert_allclose(R, [[r11, r12], [0.0, r22]], rtol=0, atol=1e-14 * r11)


@pytest.mark.parametrize("m", [64, 256, 4096, 65536])
@pytest.mark.parametrize("n,grade", [(1, 0), (7, 0), (50, 0), (50, 26)])
def test_hadamard_exact_r(m, n, grade):
    A, Rt = inputs.hadamard_exact(m, n, seed=m + n, grade_bits=grade)
    R = oracle.r_factor(A)
    # columnwise relative error (graded columns span 2^26 in magnitude)
    colerr = np.abs(R - Rt).max(axis=0) / np.abs(Rt).max(axis=0)
    assert colerr.max() < 5e-14
    assert np.array_equal(np.tril(R, -1), np.zeros_like(R))


def test_hadamard_construction_is_orthogonal():
    # guards the pin above: the generator's Q really is orthonormal
    A, Rt = inputs.hadamard_exact(256, 9, seed=3)
    Q = A @ np.linalg.inv(Rt)
    np.testing.assert_allclose(Q.T @ Q, np.eye(9), atol=1e-14)


def test_single_block_is_lapack():
    A = inputs.uniform(300, 20, 9)
    Rl = np.linalg.qr(A, mode="r")
    assert relF(oracle.r_factor(A), sign_fix(Rl)) < 1e-13


def test_gram_identity():
    A = inputs.uniform(2000, 30, 10)
    R = oracle.r_factor(A)
    G = A.T @ A
    assert np.linalg.norm(R.T @ R - G) / np.linalg.norm(A) ** 2 < 30 * 2.2e-16 * 10


def test_diagonal_nonnegative_and_upper():
    A = inputs.uniform(777, 13, 11)
    R = oracle.r_factor(A)
    assert (np.diag(R) >= 0).all() and not np.signbit(np.diag(R)).any()
    assert np.array_equal(np.tril(R, -1), np.zeros_like(R))
    assert not np.signbit(np.tril(R, -1)).any()      # +0.0, not -0.0


def test_power_of_two_scaling_bitexact():
    A = inputs.uniform(333, 9, 12)
    R = oracle.r_factor(A)
    for k in (-40, -1, 3, 60):
        assert np.array_equal(oracle.r_factor(np.ldexp(A, k)), np.ldexp(R, k))


def test_column_power_of_two_scaling_bitexact():
    A = inputs.uniform(200, 6, 13)
    d = np.ldexp(1.0, np.array([0, -3, 5, 1, -7, 2]))
    assert np.array_equal(oracle.r_factor(A * d), oracle.r_factor(A) * d)


def test_row_permutation_invariance():
    A = inputs.uniform(400, 12, 14)
    p = np.random.default_rng(0).permutation(400)
    assert relF(oracle.r_factor(A[p]), oracle.r_factor(A)) < 1e-14


# ------------------------------------------------------------ edge cases

def test_empty_and_short():
    assert oracle.r_factor(np.zeros((0, 4))).shape == (4, 4)
    assert not oracle.r_factor(np.zeros((0, 4))).any()
    assert oracle.r_factor(np.zeros((5, 0))).shape == (0, 0)
    A = inputs.uniform(3, 6, 15)           # m < n: rows m..n-1 of R are zero
    R = oracle.r_factor(A)
    assert not R[3:].any()
    np.testing.assert_allclose(R.T @ R, A.T @ A, atol=1e-14)
    assert relF(oracle.tsqr_r(A, 2), R) < 1e-14


def test_zero_column_rank_deficient():
    A = inputs.uniform(50, 4, 16)
    A[:, 2] = 0.0
    R = oracle.r_factor(A)
    assert R[2, 2] == 0.0
    np.testing.assert_allclose(R.T @ R, A.T @ A, atol=1e-13)


def test_nan_propagates():
    A = inputs.uniform(20, 3, 17)
    A[5, 1] = np.nan
    assert np.isnan(oracle.r_factor(A)).any()


# ------------------------------------------------------------ reflector

def test_reflector_definition():
    rng = np.random.default_rng(20)
    for alpha in (0.7, -0.3, 0.0, -0.0):
        x = rng.uniform(-1, 1, 6)
        beta, v, tau = oracle.reflector(alpha, x)
        y = np.concatenate([[1.0], v])
        H = np.eye(7) - tau * np.outer(y, y)
        out = H.T @ np.concatenate([[alpha], x])
        assert out[0] == pytest.approx(beta, rel=1e-15)
        assert np.abs(out[1:]).max() < 1e-15
        np.testing.assert_allclose(H @ H.T, np.eye(7), atol=1e-15)
        assert abs(beta) == pytest.approx(math.hypot(alpha, np.linalg.norm(x)), rel=1e-15)
        # beta = -sign(alpha) * norm, with the sign read from the sign bit
        assert np.signbit(beta) != np.signbit(alpha)
        assert 1.0 <= tau <= 2.0


def test_reflector_identity_when_x_zero():
    beta, v, tau = oracle.reflector(-2.5, np.zeros(4))
    assert tau == 0.0 and beta == -2.5 and not v.any()


# ------------------------------------------------------------ operator qr_uppers

def rand_upper(n, seed, scale=1.0):
    return np.triu(np.random.default_rng(seed).uniform(-1, 1, (n, n))) * scale


def test_qr_uppers_identity_element_bitexact():
    R1 = rand_upper(9, 30)
    R, V, tau = oracle.qr_uppers(R1, np.zeros((9, 9)))
    assert np.array_equal(R, R1) and not V.any() and not tau.any()


def test_qr_uppers_duplicate_is_sqrt2():
    R1 = rand_upper(12, 31)
    R, _, _ = oracle.qr_uppers(R1, R1)
    assert relF(sign_fix(R), sign_fix(R1) * math.sqrt(2.0)) < 1e-15 * 12


@pytest.mark.parametrize("c", [0.5, -3.0, 1e-8])
def test_qr_uppers_scaled_copy(c):
    R1 = rand_upper(10, 32)
    R, _, _ = oracle.qr_uppers(R1, c * R1)
    assert relF(sign_fix(R), sign_fix(R1) * math.sqrt(1.0 + c * c)) < 1e-14


def test_qr_uppers_diagonals():
    d1 = np.array([3.0, -1.0, 0.5, 2.0])
    d2 = np.array([4.0, 2.0, -1.5, 0.0])
    R, _, _ = oracle.qr_uppers(np.diag(d1), np.diag(d2))
    np.testing.assert_allclose(np.abs(R), np.diag(np.hypot(d1, d2)), rtol=1e-15, atol=0)


def test_qr_uppers_outputs_reconstruct_the_stack():
    """(R, V, tau) are the outputs named in section 3: applying the reflectors
    H_j = I - tau_j y_j y_j^T, y_j = [e_j; V(:, j)], to [R1; R2] yields [R; 0]."""
    n = 8
    R1, R2 = rand_upper(n, 33), rand_upper(n, 34)
    R, V, tau = oracle.qr_uppers(R1, R2)
    assert np.array_equal(np.tril(V, -1), np.zeros_like(V))
    W = np.vstack([R1, R2])
    for j in range(n):
        y = np.zeros(2 * n)
        y[j] = 1.0
        y[n:] = V[:, j]
        W = W - tau[j] * np.outer(y, y @ W)
    np.testing.assert_allclose(W[:n], np.triu(R), atol=1e-14)
    assert np.abs(W[n:]).max() < 1e-14
    assert np.abs(np.tril(R, -1)).max() == 0.0


def test_qr_uppers_matches_stacked_qr():
    n = 15
    R1, R2 = rand_upper(n, 35), rand_upper(n, 36)
    R, _, _ = oracle.qr_uppers(R1, R2)
    assert relF(sign_fix(R), sign_fix(np.linalg.qr(np.vstack([R1, R2]), mode="r"))) < 1e-14


def test_qr_uppers_essentially_associative_and_commutative():
    n = 11
    R1, R2, R3 = (rand_upper(n, s) for s in (40, 41, 42))
    left = oracle.qr_uppers(oracle.qr_uppers(R1, R2)[0], R3)[0]
    right = oracle.qr_uppers(R1, oracle.qr_uppers(R2, R3)[0])[0]
    assert relF(sign_fix(left), sign_fix(right)) < 1e-14
    ab = oracle.qr_uppers(R1, R2)[0]
    ba = oracle.qr_uppers(R2, R1)[0]
    assert relF(sign_fix(ab), sign_fix(ba)) < 1e-14


# ------------------------------------------------------------ method O2

@pytest.mark.parametrize("leaf", [1, 7, 50, 64, 100, 1000])
@pytest.mark.parametrize("tree", ["binary", "flat", "flat_swapped"])
def test_any_tree_any_leaf_same_r(leaf, tree):
    A = inputs.uniform(1000, 50, 50)
    assert relF(oracle.tsqr_r(A, leaf, tree), oracle.r_factor(A)) < 5e-15 * 50


def test_random_order_tree():
    A = inputs.uniform(999, 20, 51)
    P = math.ceil(999 / 64)
    perm = np.random.default_rng(1).permutation(P)
    assert relF(oracle.tsqr_r(A, 64, "order", perm), oracle.r_factor(A)) < 1e-13


def test_tsqr_hadamard_exact():
    A, Rt = inputs.hadamard_exact(4096, 50, seed=5, grade_bits=20)
    R = oracle.tsqr_r(A, 64, "binary")
    colerr = np.abs(R - Rt).max(axis=0) / np.abs(Rt).max(axis=0)
    assert colerr.max() < 5e-14


def test_cost_model():
    """Table 3's cost statement: the operator costs 2/3 n^3 against 10/3 n^3 for
    a dense Householder QR of the 2n-by-n stack; the whole method costs 2mn^2
    to leading order whatever the leaf size (sections 2 and 4)."""
    n = 200
    merge = oracle.tsqr_flops(2 * n, n, n) - 2 * oracle.tsqr_flops(n, n, n)
    assert merge / (2.0 / 3.0 * n ** 3) == pytest.approx(1.0, rel=0.03)
    assert oracle.tsqr_flops(2 * n, n, 2 * n) / (10.0 / 3.0 * n ** 3) == pytest.approx(1.0, rel=0.03)
    m = 1_000_000
    for leaf in (100, 1000, 100000):
        assert oracle.tsqr_flops(m, 50, leaf) / (2.0 * m * 50 ** 2) == pytest.approx(1.0, rel=0.03)


def test_reflector_tiny_norm_is_scale_invariant():
    """Norms below the safe minimum are handled by an exact power-of-two
    rescaling: v and tau equal those of the scaled-up vector bit for bit."""
    big = oracle.reflector(3.0, [4.0, -12.0])
    tiny = oracle.reflector(np.ldexp(3.0, -1040), np.ldexp([4.0, -12.0], -1040))
    assert tiny[2] == big[2]
    assert np.array_equal(tiny[1], big[1])
    assert tiny[0] == np.ldexp(big[0], -1040)
    assert big[0] == -13.0


def test_rank_deficient_blocks_stay_finite():
    # one-row blocks: every intermediate triangle is rank deficient
    A = inputs.uniform(300, 40, 52)
    for tree in ("binary", "flat", "flat_swapped"):
        R = oracle.tsqr_r(A, 1, tree)
        assert np.isfinite(R).all()
        assert relF(R, oracle.r_factor(A)) < 1e-13


# ---- the Q factor (definition Q = A R^-1) ------------------------------------------

@pytest.mark.parametrize("m,n,seed", [(300, 7, 3), (1000, 50, 4), (64, 64, 5), (5000, 1, 6)])
def test_q_factor_orthonormal_and_reconstructs(m, n, seed):
    A = inputs.uniform(m, n, seed)
    Q = oracle.q_factor(A)
    R = oracle.r_factor(A)
    assert Q.shape == (m, n)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) < 1e-13 * max(1.0, np.linalg.cond(A))
    assert np.linalg.norm(Q @ R - A) / np.linalg.norm(A) < 1e-14


def test_q_factor_single_column_closed_form():
    a = inputs.uniform(777, 1, 8)
    q = oracle.q_factor(a)
    np.testing.assert_allclose(q[:, 0], a[:, 0] / np.linalg.norm(a[:, 0]), rtol=0, atol=1e-16)


def test_q_factor_matches_lapack_up_to_column_signs():
    A = inputs.uniform(2000, 20, 9)
    Qn, Rn = np.linalg.qr(A)
    Q = oracle.q_factor(A)
    assert np.abs(Q - Qn * np.sign(np.diag(Rn))).max() < 1e-14


def test_q_factor_exact_for_hadamard_construction():
    # A = H R_true with H orthonormal (scaled Hadamard columns) exactly: Q = H
    A, Rt = inputs.hadamard_exact(4096, 16, seed=2)
    H = np.linalg.solve(Rt.T, A.T).T            # exact up to rounding: the scaled Hadamard columns
    Q = oracle.q_factor(A)
    assert np.abs(Q - H).max() < 1e-15 * 64
    assert set(np.unique(np.round(np.abs(H) * 64, 9))) == {1.0}


def test_q_factor_diagonal_input_is_identity_bitexact():
    d = np.array([3.0, 0.5, 7.25, 1e-3])
    Q = oracle.q_factor(np.diag(d))
    assert np.array_equal(Q, np.eye(4))


def test_q_factor_refuses_rank_deficient_and_wide_inputs():
    A = inputs.uniform(50, 4, 10)
    A[:, 2] = 0.0
    with pytest.raises(RuntimeError):
        oracle.q_factor(A)
    with pytest.raises(RuntimeError):
        oracle.q_factor(inputs.uniform(3, 5, 11))


# ---- the Gram matrix and the backward error (used as kappa-free parity gates) ----

def _exact_gram(A):
    """A^T A in exact rational arithmetic (fractions), rounded to doubles."""
    from fractions import Fraction
    F = [[Fraction(float(v)) for v in col] for col in np.asarray(A, dtype=np.float64).T]
    n = len(F)
    return np.array([[float(sum(a * b for a, b in zip(F[j], F[k]))) for k in range(n)] for j in range(n)])


def test_gram_integer_matrices_exact():
    rng = np.random.default_rng(21)
    A = rng.integers(-1000, 1000, size=(300, 7)).astype(np.float64)
    Ai = A.astype(np.int64)
    assert np.array_equal(oracle.gram(A), (Ai.T @ Ai).astype(np.float64))


def test_gram_wide_dynamic_range_is_correctly_rounded():
    """Entries spanning 2^-60 .. 2^60: the double-double sum rounds to the
    exactly rounded value of the rational sum (a plain double sum does not)."""
    rng = np.random.default_rng(22)
    A = np.ldexp(rng.uniform(-1, 1, size=(60, 4)), rng.integers(-60, 61, size=(60, 4)))
    G = oracle.gram(A)
    Ge = _exact_gram(A)
    assert np.array_equal(G, Ge)
    assert np.array_equal(G, G.T)


def test_gram_residual_zero_for_exact_construction():
    """A = Q R_true exactly with Q's columns exactly orthonormal: R_true^T
    R_true = A^T A holds exactly, and the double-double residual is exactly 0."""
    for grade in (0, 26):
        A, Rt = inputs.hadamard_exact(1024, 12, seed=23, grade_bits=grade)
        assert oracle.gram_residual(A, Rt) == 0.0
        # the strict lower triangle of R is ignored
        Rl = Rt.copy()
        Rl[5, 2] = 7.0
        assert oracle.gram_residual(A, Rl) == 0.0


def test_gram_residual_closed_form_for_one_perturbed_entry():
    """R = R_true + d e_i e_k^T changes R^T R by d (e_k r_i^T + r_i e_k^T) +
    d^2 e_k e_k^T (r_i = row i of R_true): the residual equals the norm of that
    matrix over ||A||_F^2, computed here exactly with fractions."""
    from fractions import Fraction
    A, Rt = inputs.hadamard_exact(256, 9, seed=24)
    nA2 = sum(Fraction(float(v)) ** 2 for v in A.ravel())
    for (i, k, d) in [(0, 0, 2.0 ** -20), (3, 7, -1e-9), (8, 8, 0.5)]:
        R = Rt.copy()
        R[i, k] += d
        d = Fraction(float(R[i, k])) - Fraction(float(Rt[i, k]))   # the perturbation as stored
        ri = [Fraction(float(v)) for v in Rt[i]]
        D = [[Fraction(0)] * 9 for _ in range(9)]
        for c in range(9):
            D[k][c] += d * ri[c]
            D[c][k] += d * ri[c]
        D[k][k] += d * d
        expect = math.sqrt(float(sum(x * x for row in D for x in row))) / float(nA2)
        got = oracle.gram_residual(A, R)
        assert abs(got - expect) <= 1e-12 * expect, (i, k, d, got, expect)


def test_gram_residual_is_kappa_free_and_catches_fp32():
    """The residual of an FP64 Householder R stays at the FP64 rounding level
    whatever the condition number, while an R computed in FP32 (LAPACK
    sgeqrf) sits near the FP32 rounding level: the property that makes it a
    parity gate able to reject an uncorrected FP32 factor."""
    for kappa in (1.0, 1e4, 1e8):
        A = inputs.conditioned(4096, 30, kappa, seed=25)
        A64 = A.astype(np.float64)
        r64 = oracle.gram_residual(A64, oracle.r_factor(A64))
        r32 = oracle.gram_residual(A64, np.linalg.qr(A, mode="r").astype(np.float64))
        assert r64 < 1e-15 and r32 > 1e-11, (kappa, r64, r32)


def test_parallel_check_batch_equals_serial_oracle():
    """oracle.parallel gives, bit for bit, the serial oracle's R and backward
    error for every instance of a ragged batch (including empty ones)."""
    from oracle import parallel
    n = 9
    sizes = [0, 1, 5, 9, 300, 2000]
    offsets = np.concatenate([[0], np.cumsum(np.array(sizes[:-1]) * n)])
    rng = np.random.default_rng(26)
    flat = rng.uniform(-1, 1, int(sum(sizes)) * n).astype(np.float32)
    Rt = [np.triu(rng.uniform(-1, 1, (n, n))) for _ in sizes]
    Ro, g = parallel.check_batch(flat, [(o, m, n, m) for o, m in zip(offsets, sizes)], Rt, nproc=2)
    for b, (o, m) in enumerate(zip(offsets, sizes)):
        A = flat[o:o + m * n].reshape(n, m).T.astype(np.float64)
        if m == 0:
            assert np.all(Ro[b] == 0) and g[b] == 0.0
            continue
        assert np.array_equal(Ro[b], oracle.r_factor(A)), b
        assert g[b] == oracle.gram_residual(A, Rt[b]), b


def test_threaded_method_matches_the_definition():
    """oracle.parallel.tsqr_r_threads (the method on host cores: block QRs
    in threads, then the operator over a binary tree) agrees with the
    definition to rounding, for block counts that do and do not divide m."""
    from oracle import parallel
    A = inputs.uniform(5003, 12, 27)
    Ro = oracle.r_factor(A)
    for t in (1, 2, 3, 8):
        R = parallel.tsqr_r_threads(A, t)
        assert relF(R, Ro) < 1e-14, t
        assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) >= 0), t
