"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module only draws random matrices and forms exact right-hand sides; it
holds none of the solver's multi-word arithmetic and imports neither the
product package nor the oracle (it may use torch's library GEMM for exact
products of small-integer slice matrices).

The paper's own test problem (Kouya 2021, Sec. 3: A = R D R^-1 with an
unpublished random R, x = [0..n-1]) has no published seed, so the workloads
here are seeded stand-ins with the same structure the solver is exercised on:
  * ``uniform``: entries i.i.d. uniform[-1, 1];
  * ``randsvd``: A = U diag(sigma) V^T with U, V Haar-orthogonal (QR of a
    Gaussian matrix with the R-diagonal sign fix, Mezzadri 2007) and sigma
    geometrically spaced from 1 down to 1/cond, rounded to binary64 entries;
  * ``randsvd_words``: the same product kept to about 150 bits per row in up
    to four binary64 words per entry, for condition numbers that binary64
    entries cannot carry (above about 1e15);
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


def _split(x):
    """Veltkamp split: x = hi + lo, hi with at most 26 significant bits."""
    c = 134217729.0 * x
    hi = c - (c - x)
    return hi, x - hi


def _prod_exact(a, b):
    """p + e == a * b exactly (Dekker; numpy has no fused multiply-add)."""
    p = a * b
    ah, al = _split(a)
    bh, bl = _split(b)
    e = ((ah * bh - p) + ah * bl + al * bh) + al * bl
    return p, e


def _sum_exact(a, b):
    s = a + b
    bb = s - a
    return s, (a - (s - bb)) + (b - bb)


def _exact_matmul(n: int):
    """a @ b.T for slice matrices whose every partial sum is exact in
    binary64 (so any summation order gives the same result): a library GEMM
    on the GPU when torch has one and the matrices are large, else numpy
    (also in a worker forked from a process that already uses the GPU)."""
    try:
        import torch
        bad_fork = getattr(torch.cuda, "_is_in_bad_fork", lambda: False)()
        if n >= 512 and not bad_fork and torch.cuda.is_available():
            def mm(a, b):
                ta = torch.from_numpy(a).cuda()
                tb = torch.from_numpy(b).cuda()
                return (ta @ tb.T.contiguous()).cpu().numpy()
            return mm
    except ImportError:
        pass
    return lambda a, b: a @ b.T


def randsvd_words(n: int, cond: float, g: np.random.Generator, bits: int = 150, symmetric: bool = False,
                  sigma: np.ndarray | None = None) -> np.ndarray:
    """U diag(sigma) V^T for matrices too ill-conditioned for binary64 entries
    (rounding each entry to 53 bits would perturb A by about 1e-16 ||A|| and
    cap its condition number near 1e17): the same U, V, sigma as ``randsvd``,
    the product formed to about `bits` bits below each row's scale and kept
    as up to four binary64 words per entry.  Every entry of row i is a
    multiple of one power of two 2^G_i (about 2^-`bits` times the row's
    largest possible entry), so each row sum has few enough bits for the
    quad-double right-hand side to hold it exactly.  Returns K-plane words
    (4, n, n).

    Formation: W = U diag(sigma) exactly as two words (Dekker products); W
    and V are cut into beta-bit slices on per-row grids, every slice product
    W_p V_q^T is exact in binary64 (2 (beta + 1) + log2 n <= 53 bits), the
    pairs above the target are summed, each entry rounded to the row grid
    and accumulated exactly in 50-bit integer limbs, then written back as a
    non-overlapping binary64 expansion.  ``symmetric`` takes V = U
    (A = U diag(sigma) U^T, the paper's R D R^-1 with an orthogonal R);
    ``sigma`` replaces the geometric singular values."""
    U = haar(n, g)
    V = U if symmetric else haar(n, g)
    i = np.arange(n, dtype=np.float64)
    if sigma is None:
        sigma = cond ** (-i / max(n - 1, 1))
    Whi, Wlo = _prod_exact(U, sigma[None, :])
    lg = max(1, math.ceil(math.log2(max(n, 2))))
    beta = (53 - lg) // 2 - 1
    # row scales (|x| < 2^E over the row) of W and V
    E = np.frexp(np.abs(Whi).max(axis=1))[1].astype(np.int64)
    F = np.frexp(np.abs(V).max(axis=1))[1].astype(np.int64)
    nq_w = -(-(bits + lg + 8) // beta)
    nq_v = -(-(53 + 40) // beta)

    def cut(words, scale, count):
        rem = [w.copy() for w in words]
        out = []
        for q in range(count):
            e = (scale - (q + 1) * beta)[:, None]
            sl = np.zeros_like(rem[0])
            for t in range(len(rem)):
                rho = np.ldexp(np.rint(np.ldexp(rem[t], -e)), e)
                rem[t] = rem[t] - rho
                sl = sl + rho  # exact: both on the grid 2^e, below 2^(beta + 2) units
            out.append(sl)
        return out

    Ws = cut([Whi, Wlo], E, nq_w)
    Vs = cut([V], F, nq_v)
    mm = _exact_matmul(n)
    Fmax = int(F.max())
    G = E + Fmax - bits  # row grid of A
    LB = 50
    limbs = [np.zeros((n, n), dtype=np.int64) for _ in range(5)]
    pmax = (bits + lg + 3) // beta  # pairs p + q above this stay below the grid
    for p_ in range(nq_w):
        for q_ in range(nq_v):
            if p_ + q_ > pmax:
                continue
            x = mm(Ws[p_], Vs[q_])  # W_p V_q^T, exact
            for k in range(4, 0, -1):
                sc = (G + LB * k)[:, None]
                t = np.trunc(np.ldexp(x, -sc))
                limbs[k] += t.astype(np.int64)
                x = x - np.ldexp(t, sc)
            limbs[0] += np.rint(np.ldexp(x, -G[:, None])).astype(np.int64)

    def carry():
        for k in range(4):
            c = limbs[k] >> LB
            limbs[k] -= c << LB
            limbs[k + 1] += c

    carry()  # limbs 0..3 in [0, 2^LB), the sign in limb 4 (0 or -1)
    neg = limbs[4] < 0
    for k in range(5):
        limbs[k] = np.where(neg, -limbs[k], limbs[k])
    carry()  # magnitudes: limbs 0..3 in [0, 2^LB), limb 4 zero
    if np.any(limbs[4] != 0):
        raise RuntimeError("randsvd_words: entry beyond the limb range")
    sgn = np.where(neg, -1.0, 1.0)
    terms = [sgn * np.ldexp(limbs[k].astype(np.float64), (G + LB * k)[:, None]) for k in range(4)]
    # disjoint 50-bit ranges of one sign, most significant last: exact sums
    # carried from the bottom up put the value's leading 53 bits in the top
    # word and pass what is left down; repeated on the remainder words this
    # gives a four-word expansion with each word below half an ulp of the
    # one before (every step an exact two-sum, so the value is unchanged)
    for top in range(3, 0, -1):
        for _ in range(2):
            for k in range(top):
                terms[k + 1], terms[k] = _sum_exact(terms[k + 1], terms[k])
    W4 = np.stack([terms[3], terms[2], terms[1], terms[0]])
    return np.ascontiguousarray(W4.transpose(0, 2, 1))


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


def paper_sigma(n: int) -> np.ndarray:
    """The paper's diagonal (Sec. 3): d_i = 10^(-26 (i-1)/n), i = 1..n, so
    that kappa_2(A) = 10^(26 (n-1)/n) for A = R D R^-1 with R orthogonal."""
    return 10.0 ** (-26.0 * np.arange(n, dtype=np.float64) / n)


def rhs_int(Ap: np.ndarray, xs: np.ndarray) -> tuple[np.ndarray, bool]:
    """b = A xs for integer xs (|xs| < 2^11), rounded greedily to 4 binary64
    words as in ``rhs_ones``: every word of A is cut into its top 42 bits and
    the rest (at most 11 bits), so both products with xs_j are exact binary64
    numbers and ``math.fsum`` sums them exactly.  ``exact`` as in
    ``rhs_ones``."""
    aw, n, _ = Ap.shape
    xs = np.asarray(xs, dtype=np.float64)
    assert np.all(xs == np.rint(xs)) and np.all(np.abs(xs) < 2.0 ** 11)
    m, e = np.frexp(Ap)
    hi = np.ldexp(np.trunc(np.ldexp(m, 42)), e - 42)
    lo = Ap - hi
    # word w of A(i, j) is Ap[w, j, i]
    terms = np.concatenate([(hi * xs[None, :, None]).transpose(2, 0, 1).reshape(n, aw * n),
                            (lo * xs[None, :, None]).transpose(2, 0, 1).reshape(n, aw * n)], axis=1)
    b = np.zeros((4, n))
    exact = True
    for i in range(n):
        tl = terms[i].tolist()
        ws = []
        for _ in range(4):
            ws.append(math.fsum(tl + [-v for v in ws]))
        b[:, i] = ws
        if math.fsum(tl + [-v for v in ws]) != 0.0:
            exact = False
    return b, exact


def paper_problem(n: int, instance: int = 0, config: int = 7) -> tuple[np.ndarray, np.ndarray, bool, np.ndarray]:
    """The paper's test system (Sec. 3): A = R D R^-1 with d_i = 10^(-26 (i-1)/n)
    and, here, R a Haar-orthogonal matrix (R^-1 = R^T; the paper does not
    publish its R), entries kept as quad-double words; true solution
    x = [0, 1, ..., n-1], b = A x exact in quad-double.  Returns
    (A planes (4, n, n), b (4, n), exact, x)."""
    g = rng(config, instance)
    Ap = randsvd_words(n, 0.0, g, symmetric=True, sigma=paper_sigma(n))
    xs = np.arange(n, dtype=np.float64)
    b, exact = rhs_int(Ap, xs)
    return Ap, b, exact, xs


def _batch_one(args):
    config, i, n_lo, n_hi, lc_lo, lc_hi, words_above = args
    g = rng(config, i)
    n = int(g.integers(n_lo, n_hi + 1))
    cond = float(10.0 ** g.uniform(lc_lo, lc_hi))
    if words_above is not None and cond > words_above:
        # 150 bits below each row's scale hold conditions up to ~1e45; the
        # rest get 180 (the most the 4 x 50-bit limbs of the formation
        # take with headroom), which caps the stored condition near 1e54
        Ap = randsvd_words(n, cond, g, bits=150 if cond <= 1e30 else 180)
    else:
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
          progress=None, first: int = 0, words_above: float | None = None):
    """`count` independent randsvd systems: system i draws n ~ U{n_lo..n_hi}
    and cond = 10^U(lc_lo, lc_hi) from its own seed (config, first + i), so
    the batch does not depend on the number of worker processes or on how a
    long stream is cut into batches.  A system whose cond is above
    `words_above` keeps quad-double-word entries (``randsvd_words``: a
    binary64 copy could not hold that condition); the others are binary64.
    Returns lists of A planes ((1 or 4), n, n), b (4, n), exact flags and
    conds.  `progress(done)` is called every 512 systems."""
    jobs = [(config, first + i, n_lo, n_hi, lc_lo, lc_hi, words_above) for i in range(count)]
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
    """(A planes (aw, n, n), b (4, n), exact flag) for a seeded workload;
    ``randsvd_words`` gives quad-double-word entries (aw = 4)."""
    g = rng(config, instance)
    if kind == "uniform":
        Ap = planes(uniform(n, g))
    elif kind == "randsvd":
        Ap = planes(randsvd(n, cond, g))
    elif kind == "randsvd_words":
        Ap = randsvd_words(n, cond, g)
    else:
        raise ValueError(kind)
    b, exact = rhs_ones(Ap)
    return Ap, b, exact
