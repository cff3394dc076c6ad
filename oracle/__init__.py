"""CPU oracle for the R factor of a tall-skinny QR (Langou, arXiv:1002.4250).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It wraps the plain C
file ``tsqr_oracle.c`` (IEEE double, single thread, no BLAS) through ctypes and
shares nothing with the GPU library: no source, header, table or helper.

Functions (all take and return numpy arrays; matrices are column-major n-by-n
unless stated):

* :func:`r_factor` -- the definition: R of A = QR with a non-negative diagonal
  (section 2), by Householder QR of the whole matrix.
* :func:`reflector` -- one elementary reflector (the building block of the
  operator in Table 3).
* :func:`qr_uppers` -- the reduction operator R := qr(R1, R2) with the outputs
  of section 3 / Table 3: (R, V, tau).
* :func:`tsqr_r` -- the method (section 2, Table 1): block QRs then a reduction
  tree of qr_uppers, then sign normalisation.
* :func:`normalize_signs` -- the positive-diagonal convention (section 2).
* :func:`q_factor` -- the Q that goes with that R for A of full column rank,
  by its definition Q = A R^-1 (the Q section 3 leaves implicit); m-by-n.
* :func:`gram` -- A^T A with every entry summed in double-double.
* :func:`gram_residual` -- the backward error ||R^T R - A^T A||_F / ||A||_F^2
  of a computed R, formed in double-double (every R of section 2 satisfies
  R^T R = A^T A in exact arithmetic).
* :mod:`oracle.parallel` -- the same functions over many instances in a pool
  of host processes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tsqr_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_LOCK = threading.Lock()
_LIB = None

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_int64)

TREES = {"binary": 0, "flat": 1, "flat_swapped": 2, "order": 3}


def build(force: bool = False) -> str:
    """Compile ``tsqr_oracle.c`` into ``liboracle.so`` with gcc (plain -O2,
    no fast-math, no FMA contraction) and return the library path."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", _SRC, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _LIB
    with _LOCK:
        if _LIB is None:
            lib = ctypes.CDLL(build())
            lib.oracle_reflector.argtypes = [_i64, _dp, _dp, _i64, _dp]
            lib.oracle_r_factor.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64]
            lib.oracle_q_factor.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64]
            lib.oracle_qr_uppers.argtypes = [_i64, _dp, _dp, _dp]
            lib.oracle_tsqr_r.argtypes = [_i64, _i64, _dp, _i64, _i64, ctypes.c_int, _lp, _dp, _i64]
            lib.oracle_normalize_signs.argtypes = [_i64, _dp, _i64]
            lib.oracle_normalize_signs.restype = None
            lib.oracle_tsqr_flops.argtypes = [_i64, _i64, _i64]
            lib.oracle_tsqr_flops.restype = ctypes.c_double
            lib.oracle_gram.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64]
            lib.oracle_gram_residual.argtypes = [_i64, _i64, _dp, _i64, _dp, _i64]
            lib.oracle_gram_residual.restype = ctypes.c_double
            _LIB = lib
        return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _fortran64(A) -> np.ndarray:
    A = np.asarray(A)
    if A.ndim != 2:
        raise ValueError("expected a 2-D matrix")
    return np.asfortranarray(A, dtype=np.float64)


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"{what} failed with code {rc}")


def r_factor(A) -> np.ndarray:
    """R (n-by-n, diag >= 0, exact zeros below the diagonal) of the m-by-n A."""
    A = _fortran64(A)
    m, n = A.shape
    R = np.zeros((n, n), dtype=np.float64, order="F")
    if n == 0:
        return R
    _check(_lib().oracle_r_factor(m, n, _ptr(A), max(1, m), _ptr(R), max(1, n)), "oracle_r_factor")
    return R


def q_factor(A) -> np.ndarray:
    """Q (m-by-n, orthonormal columns) of A = QR with diag(R) > 0, for A of
    full column rank (m >= n): the definition Q = A R^-1, R = r_factor(A)."""
    A = _fortran64(A)
    m, n = A.shape
    Q = np.zeros((m, n), dtype=np.float64, order="F")
    if n == 0:
        return Q
    _check(_lib().oracle_q_factor(m, n, _ptr(A), max(1, m), _ptr(Q), max(1, m)), "oracle_q_factor")
    return Q


def reflector(alpha: float, x):
    """Elementary reflector of [alpha; x]: returns (beta, v, tau) with
    (I - tau [1; v][1; v]^T)^T [alpha; x] = [beta; 0]."""
    x = np.array(x, dtype=np.float64).ravel()
    a = np.array([alpha], dtype=np.float64)
    tau = np.zeros(1, dtype=np.float64)
    xp = _ptr(x) if x.size else ctypes.cast(None, _dp)
    _check(_lib().oracle_reflector(x.size + 1, _ptr(a), xp, 1, _ptr(tau)), "oracle_reflector")
    return float(a[0]), x, float(tau[0])


def qr_uppers(R1, R2):
    """The operator of Table 3 on two n-by-n upper triangles: returns
    (R, V, tau) where R overwrote R1 and V (upper, reflectors [I; V])
    overwrote R2.  No sign normalisation."""
    R1 = _fortran64(R1).copy(order="F")
    R2 = _fortran64(R2).copy(order="F")
    n = R1.shape[0]
    if R1.shape != (n, n) or R2.shape != (n, n):
        raise ValueError("R1 and R2 must both be n-by-n")
    tau = np.zeros(max(n, 1), dtype=np.float64)
    _check(_lib().oracle_qr_uppers(n, _ptr(R1), _ptr(R2), _ptr(tau)), "oracle_qr_uppers")
    return R1, R2, tau[:n]


def tsqr_r(A, leaf_rows: int, tree: str = "binary", perm=None) -> np.ndarray:
    """The method: blocks of ``leaf_rows`` rows, local QR, reduction over
    ``tree`` ("binary", "flat", "flat_swapped" or "order" with ``perm``),
    then sign normalisation."""
    A = _fortran64(A)
    m, n = A.shape
    R = np.zeros((n, n), dtype=np.float64, order="F")
    if n == 0:
        return R
    kind = TREES[tree]
    if kind == 3:
        perm = np.ascontiguousarray(perm, dtype=np.int64)
        pp = perm.ctypes.data_as(_lp)
    else:
        pp = ctypes.cast(None, _lp)
    _check(_lib().oracle_tsqr_r(m, n, _ptr(A), max(1, m), int(leaf_rows), kind, pp, _ptr(R), max(1, n)),
           "oracle_tsqr_r")
    return R


def normalize_signs(R) -> np.ndarray:
    """Copy of R with every row whose diagonal sign bit is set negated."""
    R = _fortran64(R).copy(order="F")
    n = R.shape[0]
    _lib().oracle_normalize_signs(n, _ptr(R), max(1, n))
    return R


def tsqr_flops(m: int, n: int, leaf_rows: int) -> float:
    """Flop count of :func:`tsqr_r` in the paper's cost model."""
    return float(_lib().oracle_tsqr_flops(m, n, leaf_rows))


def gram(A) -> np.ndarray:
    """A^T A (n-by-n), every entry summed in double-double from exact
    products and rounded once."""
    A = _fortran64(A)
    m, n = A.shape
    G = np.zeros((n, n), dtype=np.float64, order="F")
    if n == 0:
        return G
    _check(_lib().oracle_gram(m, n, _ptr(A), max(1, m), _ptr(G), max(1, n)), "oracle_gram")
    return G


def gram_residual(A, R) -> float:
    """||R^T R - A^T A||_F / ||A||_F^2 for the m-by-n A and the n-by-n upper
    triangle of R (its strict lower part is ignored), formed in double-double:
    the backward error of R as a QR factor of A.  Independent of the condition
    number of A, unlike the forward error of R."""
    A = _fortran64(A)
    R = _fortran64(R)
    m, n = A.shape
    if R.shape != (n, n):
        raise ValueError("R must be n-by-n")
    if n == 0 or m == 0:
        return 0.0
    v = float(_lib().oracle_gram_residual(m, n, _ptr(A), max(1, m), _ptr(R), max(1, n)))
    if v < 0:
        raise ValueError("gram_residual: A is zero or sizes are invalid")
    return v
