"""Seeded synthetic inputs shaped like the paper's workloads.

The paper measures a tall-skinny matrix with m = 1,000,000 rows and n = 50
columns in double precision (section 4, Table 2) and does not say what the
entries are.  These generators stand in for that data; they hold none of the
factorisation's arithmetic and are shared by the tests, the benchmark and the
smoke check, so both the GPU path and the oracle see the same bits.

All matrices are returned column-major (``numpy`` Fortran order): element
(i, j) of an m-by-n matrix is entry ``i + j*m`` of the underlying buffer.
Float32 inputs are the round-to-nearest-even rounding of the float64 draws.
"""
from __future__ import annotations

import math

import numpy as np


def uniform(m: int, n: int, seed: int, dtype=np.float64) -> np.ndarray:
    """i.i.d. uniform[-1, 1) entries, drawn by ``numpy.random.default_rng(seed)``
    in column-major order (the first m draws are column 0)."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, size=m * n)
    A = a.reshape(n, m).T
    if np.dtype(dtype) == np.float32:
        A = A.astype(np.float32)
    return np.asfortranarray(A)


def _is_power_of_4(m: int) -> bool:
    return m >= 1 and (m & (m - 1)) == 0 and (m.bit_length() - 1) % 2 == 0


def hadamard_exact(m: int, n: int, seed: int = 0, grade_bits: int = 0):
    """A matrix whose exact R is known: returns ``(A, R_true)``.

    Q is the first n columns of the Sylvester-Hadamard matrix of order m
    (entry (i, j) = (-1)^popcount(i & j)) divided by sqrt(m); for m a power of 4
    sqrt(m) is a power of two, so Q has exactly orthonormal columns in binary64.
    R_true is upper triangular with diagonal 64 and off-diagonal integers drawn
    uniformly from [-3, 3] (``default_rng(seed)``), then column j is scaled by
    2^-e_j with e_j = round(j * grade_bits / (n - 1)), which sets the condition
    number to about 2^grade_bits without losing exactness.  A = Q R_true is
    computed exactly (integer partial sums below 2^53, power-of-two scalings), so
    the R factor of A with a positive diagonal is exactly R_true.
    """
    if not _is_power_of_4(m):
        raise ValueError("m must be a power of 4")
    if n > m:
        raise ValueError("need n <= m")
    rng = np.random.default_rng(seed)
    Rt = np.triu(rng.integers(-3, 4, size=(n, n)).astype(np.float64), 1) + 64.0 * np.eye(n)
    if grade_bits and n > 1:
        e = np.rint(np.arange(n) * grade_bits / (n - 1)).astype(np.int64)
        Rt = Rt * np.ldexp(1.0, -e)[None, :]
    i = np.arange(m, dtype=np.int64)[:, None]
    j = np.arange(n, dtype=np.int64)[None, :]
    S = np.where(np.bitwise_count(i & j) % 2 == 0, 1.0, -1.0)
    half = (m.bit_length() - 1) // 2
    A = np.asfortranarray(np.ldexp(S @ Rt, -half))
    return A, np.asfortranarray(Rt)


def pad_rows(A: np.ndarray, m_new: int) -> np.ndarray:
    """A with zero rows appended up to m_new rows (zero rows leave R unchanged)."""
    m, n = A.shape
    out = np.zeros((m_new, n), dtype=A.dtype, order="F")
    out[:m] = A
    return out


def batched_sizes(count: int = 4096, lo: int = 64, hi: int = 65536, seed: int = 2) -> np.ndarray:
    """Row counts m_b = floor(exp(U[ln lo, ln hi))) from ``default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    return np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), size=count))).astype(np.int64)


def batched_instance(b: int, m: int, n: int = 50, seed: int = 2, dtype=np.float32) -> np.ndarray:
    """Entries of instance b of a ragged batch: m-by-n uniform[-1, 1) from
    ``default_rng([seed, b])`` in column-major order (Fortran array), so any
    instance can be regenerated on its own."""
    rng = np.random.default_rng([seed, b])
    a = rng.uniform(-1.0, 1.0, size=m * n)
    if np.dtype(dtype) == np.float32:
        a = a.astype(np.float32)
    return np.asfortranarray(a.reshape(n, m).T)


def batched_uniform(count: int = 4096, n: int = 50, lo: int = 64, hi: int = 65536, seed: int = 2,
                    dtype=np.float32):
    """Ragged batch: the sizes of :func:`batched_sizes`, the entries of
    instance b from :func:`batched_instance`, each instance an m_b-by-n
    column-major block, blocks concatenated in instance order.  Returns
    ``(flat, sizes, offsets)`` with ``offsets[b]`` the element offset of
    instance b."""
    sizes = batched_sizes(count, lo, hi, seed)
    offsets = np.zeros(count, dtype=np.int64)
    np.cumsum(sizes[:-1] * n, out=offsets[1:])
    total = int(sizes.sum()) * n
    flat = np.empty(total, dtype=np.dtype(dtype))
    for b in range(count):
        m = int(sizes[b])
        o = int(offsets[b])
        flat[o:o + m * n] = batched_instance(b, m, n, seed, dtype).T.ravel()
    return flat, sizes, offsets


def instance(flat: np.ndarray, sizes, offsets, b: int, n: int) -> np.ndarray:
    """View of instance b of a ragged batch as an m_b-by-n Fortran array."""
    m = int(sizes[b])
    o = int(offsets[b])
    return flat[o:o + m * n].reshape(n, m).T


def conditioned(m: int, n: int, kappa: float, seed: int, dtype=np.float32) -> np.ndarray:
    """A = U diag(sigma) V^T with singular values sigma_j = kappa^(-j/(n-1))
    (so cond_2(A) = kappa before rounding), U (m x n) and V (n x n) the
    orthonormal factors of uniform[-1, 1) draws from ``default_rng(seed)``,
    formed in FP64 and rounded to ``dtype``.  Column-major."""
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.uniform(-1.0, 1.0, size=(m, n)))
    V, _ = np.linalg.qr(rng.uniform(-1.0, 1.0, size=(n, n)))
    sigma = kappa ** (-np.arange(n) / max(n - 1, 1))
    A = (U * sigma[None, :]) @ V.T
    return np.asfortranarray(A.astype(dtype))


def conditioned_batch(batch: int, m: int, n: int, log10_kappa_max: float = 8.0, seed: int = 3,
                      dtype=np.float32):
    """Instances i = 0..batch-1 of :func:`conditioned` with
    kappa_i = 10^(log10_kappa_max * i / (batch - 1)) and seed (seed, i),
    stacked with stride m*n in one flat array.  Returns (flat, kappas)."""
    kappas = 10.0 ** (log10_kappa_max * np.arange(batch) / max(batch - 1, 1))
    flat = np.empty(batch * m * n, dtype=dtype)
    for i in range(batch):
        A = conditioned(m, n, float(kappas[i]), seed=[seed, i], dtype=dtype)
        flat[i * m * n:(i + 1) * m * n] = A.T.ravel()
    return flat, kappas


def conditioned_batch_device(torch, batch: int, m: int, n: int, log10_kappa_max: float = 8.0, seed: int = 0,
                             device="cuda"):
    """A device-side counterpart of :func:`conditioned_batch` for large
    training sets: A_i = G_i diag(sigma_i) V_i^T with G_i (m x n) standard
    normal draws from a device generator seeded with ``seed`` (so cond_2(A_i)
    is kappa_i times cond_2(G_i), about 1 + 2 sqrt(n/m)), V_i the orthonormal
    factor of CPU normal draws from a generator seeded with ``seed``, sigma_j =
    kappa_i^(-j/(n-1)) and kappa_i = 10^(log10_kappa_max i/(batch-1)), formed
    in FP32.  Returns (flat FP32 device tensor, instance i column-major at
    i*m*n; kappas as a numpy array)."""
    kappas = 10.0 ** (log10_kappa_max * np.arange(batch) / max(batch - 1, 1))
    gc = torch.Generator(device="cpu")
    gc.manual_seed(int(seed))
    V, _ = torch.linalg.qr(torch.randn((batch, n, n), generator=gc, dtype=torch.float64))
    sig = torch.from_numpy(kappas[:, None] ** (-np.arange(n)[None, :] / max(n - 1, 1)))
    Vs = (V * sig[:, None, :]).to(device=device, dtype=torch.float32)
    gd = torch.Generator(device=device)
    gd.manual_seed(int(seed))
    Gt = torch.randn((batch, n, m), generator=gd, device=device, dtype=torch.float32)
    # row c of instance i's A^T = V diag(sigma) G^T is column c of A_i
    At = torch.bmm(Vs, Gt)
    del Gt
    return At.reshape(-1), kappas
