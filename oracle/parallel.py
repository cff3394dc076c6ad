"""The oracle over many instances at once, in a pool of host processes.

TEST INFRASTRUCTURE ONLY (same rule as the rest of ``oracle``).  The oracle is
single-threaded C, so checking every instance of a large batch (thousands of
matrices, tens of millions of rows) is spread over worker processes.  Each
instance is sent to a worker as its own array (at most a few instances are in
flight at once, so memory stays near one copy of the batch); the worker
computes the oracle's R (the definition of section 2) and the backward error
of the R under test.  Workers are started with ``spawn``, so a parent that has
initialised a GPU never forks it.

The input generators of ``paper_1002_4250_amd.inputs`` lay a batch out as one
flat array: instance b is an m_b-by-n column-major block at element offset
o_b with leading dimension lda_b.
"""
from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np


def _work(args):
    """(index, R_oracle, gram_residual(A, R_test)) for one instance."""
    import oracle
    b, A, R_test = args
    m, n = A.shape
    if m == 0 or n == 0:
        return b, np.zeros((n, n)), 0.0
    A = np.asfortranarray(A, dtype=np.float64)
    Ro = oracle.r_factor(A)
    g = oracle.gram_residual(A, R_test) if R_test is not None else float("nan")
    return b, Ro, g


def workers(limit: int = 16) -> int:
    """Worker count: the host's CPUs, at most ``limit``."""
    return max(1, min(limit, os.cpu_count() or 1))


def _jobs(flat, instances, R_test):
    for b, (off, m, n, lda) in enumerate(instances):
        off, m, n, lda = int(off), int(m), int(n), int(lda)
        if m == 0 or n == 0:
            A = np.zeros((m, n), dtype=flat.dtype)
        else:
            A = np.lib.stride_tricks.as_strided(flat[off:], shape=(m, n),
                                                strides=(flat.itemsize, flat.itemsize * lda)).copy(order="F")
        rt = None if R_test is None else np.asfortranarray(R_test[b], dtype=np.float64)
        yield b, A, rt


def check_batch(flat: np.ndarray, instances, R_test=None, nproc: int | None = None):
    """Run the oracle on every instance of a flat batch.

    ``instances`` is a sequence of (offset, m, n, lda); ``R_test`` an optional
    sequence of n-by-n matrices (the results under test) whose backward error
    against their instance is computed too.  Returns (list of oracle R, array
    of backward errors, NaN where no R_test was given)."""
    flat = np.asarray(flat).ravel()
    Ro = [None] * len(instances)
    g = np.full(len(instances), np.nan)
    ctx = mp.get_context("spawn")
    with ctx.Pool(nproc or workers()) as pool:
        for b, r, res in pool.imap_unordered(_work, _jobs(flat, instances, R_test), chunksize=1):
            Ro[b] = r
            g[b] = res
    return Ro, g


def tsqr_r_threads(A, threads: int) -> np.ndarray:
    """The paper's method on host cores: the rows of A split into `threads`
    contiguous blocks, each block's R by the oracle's definition in its own
    thread (the C code runs without the interpreter lock), then the block
    triangles combined pairwise with the oracle's operator qr_uppers over a
    binary tree (lower block on top), and the signs normalized (section 2).
    A baseline for the GPU, not a reference: its result agrees with
    ``oracle.r_factor`` to rounding."""
    import concurrent.futures as cf

    import oracle
    A = np.asarray(A)
    m, n = A.shape
    threads = max(1, min(int(threads), max(1, m // max(n, 1))))
    bounds = [m * i // threads for i in range(threads + 1)]
    with cf.ThreadPoolExecutor(max_workers=threads) as pool:
        tris = list(pool.map(lambda i: oracle.r_factor(A[bounds[i]:bounds[i + 1]]), range(threads)))
    while len(tris) > 1:
        nxt = []
        for i in range(0, len(tris) - 1, 2):
            R, _, _ = oracle.qr_uppers(tris[i], tris[i + 1])
            nxt.append(np.triu(R))
        if len(tris) % 2:
            nxt.append(tris[-1])
        tris = nxt
    return oracle.normalize_signs(tris[0])
