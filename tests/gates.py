"""Parity gates shared by the GPU tests (numpy only; no oracle arithmetic).

Three measures of how far a computed R is from the oracle's, two of which
stay meaningful at any condition number kappa:

* relF  -- ||R - R_oracle||_F / ||R_oracle||_F, the global forward error.  It
  is dominated by the leading rows of R, so at high kappa the small trailing
  rows can be wholly wrong without moving it; its gates grow with kappa.
* backward error -- ||R^T R - A^T A||_F / ||A||_F^2 (``oracle.gram_residual``,
  formed in double-double).  A backward-stable QR in unit roundoff u meets it
  at c n u whatever kappa is; an R computed in FP32 sits near the FP32
  rounding level.  Gates: 1e-14 (about 2 n u_64 at n = 50) for FP64 results,
  1e-6 for FP32 results.
* row-scaled error -- max over rows i of ||R_i - R_oracle,i|| / ||R_oracle,i||,
  which sees every row, however small.  Two FP64 backward-stable
  factorizations (LAPACK dgeqrf against the oracle) differ by at most about
  3e-11 at kappa = 1e8 on the conditioned inputs, growing roughly like
  kappa^0.55, while an FP32 factor sits near 4e-8 at every kappa; the gate
  1e-14 * max(1, kappa)^0.6 passes the first with a margin of about 20 and
  rejects the second from kappa = 1e2 up.
"""
import numpy as np

GRAM64 = 1e-14
GRAM32 = 1e-6


def relF(X, Y):
    return float(np.linalg.norm(X - Y) / max(np.linalg.norm(Y), 1e-300))


def row_scaled(X, Y):
    """max_i ||X_i - Y_i|| / ||Y_i|| over the rows of Y with a nonzero norm."""
    ny = np.linalg.norm(Y, axis=1)
    keep = ny > 0
    if not np.any(keep):
        return 0.0
    return float(np.max(np.linalg.norm(X - Y, axis=1)[keep] / ny[keep]))


def row_gate64(kappa):
    return 1e-14 * max(1.0, float(kappa)) ** 0.6


def kappa_of(R):
    """2-norm condition number of an upper triangle (that of A, since A = QR)."""
    s = np.linalg.svd(R, compute_uv=False)
    return float(s[0] / s[-1]) if s[-1] > 0 else float("inf")
