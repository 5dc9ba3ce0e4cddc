"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random matrices and forms exact right-hand sides; it
holds none of the solver's multi-word arithmetic and imports neither the
product package nor the oracle.

The paper's own test problem (Kouya 2021, Sec. 3: A = R D R^-1 with an
unpublished random R, x = [0..n-1]) has no published seed, so the workloads
here are seeded stand-ins with the same structure the solver is exercised on:
  * ``uniform``: entries i.i.d. uniform[-1, 1];
  * ``randsvd``: A = U diag(sigma) V^T with U, V Haar-orthogonal (QR of a
    Gaussian matrix with the R-diagonal sign fix, Mezzadri 2007) and sigma
    geometrically spaced from 1 down to 1/cond, rounded to binary64 entries;
  * right-hand side b = A * ones computed exactly and rounded to canonical
    quad-double words, so the exact solution of the stored system is all
    ones whenever the rounding is exact (reported as ``exact``).
Seeds: numpy PCG64(2107_12550 + 1000 * config + instance).
Layout: a K-word matrix is a float64 array (K, n, n) with [w, j, i] = word w
of entry (i, j); a K-word vector is (K, n).
"""
from __future__ import annotations

import math

import numpy as np

SEED_BASE = 2107_12550


def rng(config: int, instance: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + 1000 * config + instance))


def uniform(n: int, g: np.random.Generator) -> np.ndarray:
    """Dense n x n binary64 matrix, entries i.i.d. uniform[-1, 1] (row-major)."""
    return g.uniform(-1.0, 1.0, size=(n, n))


def haar(n: int, g: np.random.Generator) -> np.ndarray:
    """Haar-distributed orthogonal matrix (Mezzadri 2007)."""
    Z = g.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def randsvd(n: int, cond: float, g: np.random.Generator) -> np.ndarray:
    """U diag(sigma) V^T, sigma_i = cond^(-i/(n-1)), rounded to binary64."""
    U = haar(n, g)
    V = haar(n, g)
    i = np.arange(n, dtype=np.float64)
    sigma = cond ** (-i / max(n - 1, 1))
    return (U * sigma) @ V.T


def planes(A: np.ndarray) -> np.ndarray:
    """Row-major binary64 matrix -> one-word K-plane array (1, n, n)."""
    return np.ascontiguousarray(A.T)[None, :, :].copy()


def rhs_ones(Ap: np.ndarray) -> tuple[np.ndarray, bool]:
    """b = A * ones, exact row sums rounded greedily to 4 binary64 words
    (w0 = RN(s), w1 = RN(s - w0), ...) with ``math.fsum``, which returns the
    correctly rounded value of an exact sum.  ``exact`` is True when the four
    words represent every row sum exactly (then x* = ones exactly).
    Ap: K-plane array (aw, n, n)."""
    aw, n, _ = Ap.shape
    b = np.zeros((4, n))
    exact = True
    # row i of A = entries Ap[w, :, i] over all words w and columns
    rows = np.ascontiguousarray(Ap.transpose(2, 0, 1).reshape(n, aw * n))
    for i in range(n):
        terms = rows[i].tolist()
        ws = []
        for _ in range(4):
            w = math.fsum(terms + [-v for v in ws])
            ws.append(w)
        b[:, i] = ws
        if math.fsum(terms + [-v for v in ws]) != 0.0:
            exact = False
    return b, exact


def _batch_one(args):
    config, i, n_lo, n_hi, lc_lo, lc_hi = args
    g = rng(config, i)
    n = int(g.integers(n_lo, n_hi + 1))
    cond = float(10.0 ** g.uniform(lc_lo, lc_hi))
    Ap = planes(randsvd(n, cond, g))
    b, exact = rhs_ones(Ap)
    return Ap, b, exact, cond


def _one_blas_thread():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def batch(count: int, n_lo: int, n_hi: int, lc_lo: float, lc_hi: float, config: int = 3, workers: int = 1,
          progress=None, first: int = 0):
    """`count` independent randsvd systems: system i draws n ~ U{n_lo..n_hi}
    and cond = 10^U(lc_lo, lc_hi) from its own seed (config, first + i), so
    the batch does not depend on the number of worker processes or on how a
    long stream is cut into batches.  Returns lists of A planes (1, n, n),
    b (4, n), exact flags and conds.  `progress(done)` is called every 512
    systems."""
    jobs = [(config, first + i, n_lo, n_hi, lc_lo, lc_hi) for i in range(count)]
    out = []
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers, initializer=_one_blas_thread) as pool:
            for o in pool.imap(_batch_one, jobs, chunksize=16):
                out.append(o)
                if progress and len(out) % 512 == 0:
                    progress(len(out))
    else:
        for j in jobs:
            out.append(_batch_one(j))
            if progress and len(out) % 512 == 0:
                progress(len(out))
    return [o[0] for o in out], [o[1] for o in out], [o[2] for o in out], [o[3] for o in out]


def problem(kind: str, n: int, config: int, instance: int = 0, cond: float = 1e3):
    """(A planes (1, n, n), b (4, n), exact flag) for a seeded workload."""
    g = rng(config, instance)
    if kind == "uniform":
        A = uniform(n, g)
    elif kind == "randsvd":
        A = randsvd(n, cond, g)
    else:
        raise ValueError(kind)
    Ap = planes(A)
    b, exact = rhs_ones(Ap)
    return Ap, b, exact
