"""Brute-force R factor in high precision, for tiny inputs.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The R of A = QR with a
positive diagonal is also the upper Cholesky factor of the Gram matrix A^T A
(R^T R = A^T Q^T Q R = A^T A, section 2's uniqueness of R once the diagonal
sign is fixed).  Here A^T A is formed exactly in rational arithmetic from the
binary64 entries of A, and the Cholesky factor is taken with mpmath at a
working precision far beyond double, so the result is the exact R of the given
floating-point A to about 1e-40 relative.  Cost O(m n^2) rationals: keep
m <= 64 and n <= 8.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath
import numpy as np


def gram_exact(A):
    """A^T A as a list of lists of Fractions (exact)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    cols = [[Fraction(float(A[i, j])) for i in range(m)] for j in range(n)]
    return [[sum((cols[j][i] * cols[k][i] for i in range(m)), Fraction(0)) for k in range(n)]
            for j in range(n)]


def r_factor_mp(A, dps: int = 60):
    """Upper Cholesky factor of the exact Gram matrix, as an mpmath matrix
    (n-by-n).  Raises ValueError if A does not have full column rank."""
    G = gram_exact(A)
    n = len(G)
    with mpmath.workdps(dps):
        R = mpmath.zeros(n, n)
        for j in range(n):
            d = mpmath.mpf(G[j][j].numerator) / G[j][j].denominator
            for i in range(j):
                d -= R[i, j] ** 2
            if d <= 0:
                raise ValueError("A is rank deficient")
            R[j, j] = mpmath.sqrt(d)
            for k in range(j + 1, n):
                s = mpmath.mpf(G[j][k].numerator) / G[j][k].denominator
                for i in range(j):
                    s -= R[i, j] * R[i, k]
                R[j, k] = s / R[j, j]
        return R


def r_factor(A, dps: int = 60) -> np.ndarray:
    """:func:`r_factor_mp` rounded to float64."""
    R = r_factor_mp(A, dps)
    n = R.rows
    return np.array([[float(R[i, j]) for j in range(n)] for i in range(n)], dtype=np.float64)
