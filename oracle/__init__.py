"""ORACLE -- test infrastructure, not part of the product path.

A plain, slow CPU reference for the solver: K-word (binary64, double-double,
triple-double, quad-double) LU with partial pivoting, substitutions, the exact
residual, and the mixed-precision iterative refinement loop of the paper's
Listing 1 (Kouya 2021, Sec. 2).  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It
shares no code with ``paper_2107_12550_amd``; both sides read the same seeded
inputs from ``synth``.

Arrays use the K-plane layout: a K-word n x n matrix is a float64 array of
shape (K, n, n) whose element [w, j, i] is word w of entry (i, j) (each plane
column-major); a K-word vector is shape (K, n).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mwla.c")
_LIB = os.path.join(_HERE, "libmwla_oracle.so")
GCC_FLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC"]

# refinement status codes (same numbering as the product's C-ABI)
CONVERGED, MAX_ITER, SINGULAR, NONFINITE, STAGNATED = 0, 1, 2, 3, 5


def build() -> str:
    """Compile the C oracle with gcc (no contraction, no fast-math)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", *GCC_FLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(ctypes.c_double)
        I64 = ctypes.c_int64
        L.orc_two_sum.argtypes = [I64, P, P, P, P]
        L.orc_two_prod.argtypes = [I64, P, P, P, P]
        L.orc_fms_vec.argtypes = [ctypes.c_int, I64, P, P, P, P]
        L.orc_mul_vec.argtypes = [ctypes.c_int, I64, P, P, P]
        L.orc_add_vec.argtypes = [ctypes.c_int, I64, P, P, P]
        L.orc_recip_vec.argtypes = [ctypes.c_int, I64, P, P]
        L.orc_round_vec.argtypes = [ctypes.c_int, ctypes.c_int, I64, P, P]
        L.orc_key_gt_vec.argtypes = [ctypes.c_int, I64, P, P, ctypes.POINTER(ctypes.c_int32)]
        L.orc_getrf.argtypes = [ctypes.c_int, I64, P, I64, I64, ctypes.POINTER(I64)]
        L.orc_getrf.restype = I64
        L.orc_getrs.argtypes = [ctypes.c_int, I64, I64, P, I64, I64, ctypes.POINTER(I64), P, I64, I64]
        L.orc_residual.argtypes = [I64, ctypes.c_int, ctypes.c_int, P, I64, I64, P, I64, P, I64, P, I64]
        L.orc_residual.restype = I64
        L.orc_exact_dot.argtypes = [ctypes.c_int, I64, P, P, ctypes.POINTER(ctypes.c_int32), P]
        L.orc_exact_dot.restype = ctypes.c_int
        L.orc_oz_slices.argtypes = [ctypes.c_int, ctypes.c_int, I64, P, ctypes.c_int32, P, P]
        L.orc_oz_scale.argtypes = [I64, P]
        L.orc_oz_scale.restype = ctypes.c_int32
        L.orc_gemm.argtypes = [ctypes.c_int, I64, I64, I64, P, I64, I64, P, I64, I64, P, I64, I64]
        L.orc_oz_beta.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_oz_beta.restype = ctypes.c_int
        L.orc_oz_emin.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_oz_emin.restype = ctypes.c_int
        L.orc_oz_update.argtypes = [ctypes.c_int, ctypes.c_int, I64, I64, I64, P, I64, I64, P, I64, I64,
                                    P, I64, I64, P]
        L.orc_oz_update.restype = ctypes.c_int
        L.orc_getrf_ozaki.argtypes = [ctypes.c_int, I64, P, I64, I64, ctypes.POINTER(I64), I64, ctypes.c_int]
        L.orc_getrf_ozaki.restype = I64
        L.orc_set_threads.argtypes = [ctypes.c_int]
        L.orc_set_threads.restype = ctypes.c_int
        L.orc_get_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> int:
    """Threads the oracle's loops over independent columns and rows use
    (n < 1: the OpenMP default); returns the number in effect.  Results do
    not depend on it."""
    return int(lib().orc_set_threads(int(n)))


def threads() -> int:
    return int(lib().orc_get_threads())


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# error-free transformations and K-word primitives (vectorised, word-major)
# --------------------------------------------------------------------------

def two_sum(a, b):
    a, b = _c(a).ravel(), _c(b).ravel()
    s, e = np.empty_like(a), np.empty_like(a)
    lib().orc_two_sum(a.size, _p(a), _p(b), _p(s), _p(e))
    return s, e


def two_prod(a, b):
    a, b = _c(a).ravel(), _c(b).ravel()
    p, e = np.empty_like(a), np.empty_like(a)
    lib().orc_two_prod(a.size, _p(a), _p(b), _p(p), _p(e))
    return p, e


def fms(K: int, c, a, b) -> np.ndarray:
    """c - a*b for (K, n) arrays of K-word values."""
    c, a, b = _c(c), _c(a), _c(b)
    out = np.empty_like(a)
    lib().orc_fms_vec(K, a.shape[1], _p(c), _p(a), _p(b), _p(out))
    return out


def mul(K: int, a, b) -> np.ndarray:
    a, b = _c(a), _c(b)
    out = np.empty_like(a)
    lib().orc_mul_vec(K, a.shape[1], _p(a), _p(b), _p(out))
    return out


def add(K: int, a, b) -> np.ndarray:
    a, b = _c(a), _c(b)
    out = np.empty_like(a)
    lib().orc_add_vec(K, a.shape[1], _p(a), _p(b), _p(out))
    return out


def recip(K: int, a) -> np.ndarray:
    a = _c(a)
    out = np.empty_like(a)
    lib().orc_recip_vec(K, a.shape[1], _p(a), _p(out))
    return out


def round_words(K: int, src) -> np.ndarray:
    """Renormalise m-word values (shape (m, n), m <= 8) to K <= 8 words."""
    src = _c(src)
    m, n = src.shape
    out = np.empty((K, n))
    lib().orc_round_vec(K, m, n, _p(src), _p(out))
    return out


def key_gt(K: int, a, b) -> np.ndarray:
    a, b = _c(a), _c(b)
    out = np.empty(a.shape[1], dtype=np.int32)
    lib().orc_key_gt_vec(K, a.shape[1], _p(a), _p(b), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return out.astype(bool)


def exact_round(K: int, p, q=None, signs=None) -> tuple[np.ndarray, bool]:
    """Exact sum_t s_t p_t q_t (or sum_t s_t p_t) rounded to K canonical words."""
    p = _c(p).ravel()
    qq = None if q is None else _c(q).ravel()
    s = np.ones(p.size, dtype=np.int32) if signs is None else np.ascontiguousarray(signs, dtype=np.int32)
    out = np.zeros(K)
    bad = lib().orc_exact_dot(K, p.size, _p(p), None if qq is None else _p(qq),
                              s.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), _p(out))
    return out, bool(bad)


# --------------------------------------------------------------------------
# LU, substitutions, exact residual
# --------------------------------------------------------------------------

def stage(K: int, A: np.ndarray) -> np.ndarray:
    """Short-precision copy of an aw-word matrix (shape (aw, n, n)) in K words."""
    aw, n, _ = A.shape
    return round_words(K, A.reshape(aw, n * n)).reshape(K, n, n)


def getrf(K: int, A: np.ndarray):
    """In-place-style PA = LU of a (K, n, n) array; returns (LU, ipiv, info)."""
    LU = _c(A).copy()
    n = LU.shape[1]
    ipiv = np.zeros(n, dtype=np.int64)
    info = lib().orc_getrf(K, n, _p(LU), n, n * n, ipiv.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return LU, ipiv, int(info)


# --------------------------------------------------------------------------
# trailing update by error-free splitting (Ozaki scheme; not in the paper)
# --------------------------------------------------------------------------

OZ_SMAX = 16   # most slices
OZ_KBMAX = 64  # widest panel for which the group sums stay exact


def oz_beta(K: int, s: int) -> int:
    """Bits per slice for K-word values cut into s slices: the widest slice
    (at most 26 bits) for which every group sum of a depth-64 update stays
    below 2^53 units of its grid, so that it is exact."""
    b = int(lib().orc_oz_beta(K, s))
    if b < 0:
        raise ValueError("oz_beta: K or s out of range")
    return b


def oz_scale(x0) -> int:
    """Smallest E with |x| < 2^E for every value of x0 (0 if all zero)."""
    x0 = _c(x0).ravel()
    return int(lib().orc_oz_scale(x0.size, _p(x0)))


def oz_slices(K: int, s: int, x, E: int):
    """Cut m K-word values x (shape (K, m)) into s slices on the grids
    2^(E - (q+1) beta), beta = oz_beta(K, s); returns (slices (s, m),
    remainders (K, m))."""
    x = _c(x)
    m = x.shape[1]
    sl = np.empty((s, m))
    rem = np.empty((K, m))
    lib().orc_oz_slices(K, s, m, _p(x), E, _p(sl), _p(rem))
    return sl, rem


def oz_update(K: int, s: int, L, U, C):
    """C - L U by the split scheme.  L (K, kb, m) and U (K, nc, kb) and C
    (K, nc, m) are K-plane (column-major) blocks.  Returns (C_new, acc) with
    acc[d, j, i] the exact group sum of diagonal d."""
    L, U = _c(L), _c(U)
    C = _c(C).copy()
    _, kb, m = L.shape
    nc = U.shape[1]
    acc = np.empty((s, nc, m))
    rc = lib().orc_oz_update(K, s, m, nc, kb, _p(L), m, kb * m, _p(U), kb, nc * kb, _p(C), m, nc * m, _p(acc))
    if rc < 0:
        raise ValueError("oz_update: kb or s out of range")
    return C, acc


def oz_emin(K: int, s: int) -> int:
    """Smallest nonzero row/column scale for which the split scheme with s
    slices keeps every slice and product grid at 2^-1022 or above."""
    return int(lib().orc_oz_emin(K, s))


def getrf_ozaki(K: int, A: np.ndarray, s: int, nb: int = 64):
    """Blocked PA = LU (panel width nb) whose trailing updates use the split
    scheme with s slices; returns (LU, ipiv, info), info = -3 when a
    nonsingular factorisation met a row of L21 or column of U12 whose scale
    is below oz_emin(K, s) (the scheme was not exact there)."""
    LU = _c(A).copy()
    n = LU.shape[1]
    ipiv = np.zeros(n, dtype=np.int64)
    info = lib().orc_getrf_ozaki(K, n, _p(LU), n, n * n, ipiv.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nb, s)
    if info == -2:
        raise ValueError("getrf_ozaki: nb or s out of range")
    return LU, ipiv, int(info)


def getrs(K: int, LU: np.ndarray, ipiv: np.ndarray, b: np.ndarray) -> np.ndarray:
    """x with A x = b from the factors; b has shape (K, n) or (K, nrhs, n)."""
    LU = _c(LU)
    n = LU.shape[1]
    B = _c(b).copy()
    nrhs = 1 if B.ndim == 2 else B.shape[1]
    ipiv = np.ascontiguousarray(ipiv, dtype=np.int64)
    lib().orc_getrs(K, n, nrhs, _p(LU), n, n * n, ipiv.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                    _p(B), n, n * nrhs)
    return B


def gemm(K: int, A: np.ndarray, B: np.ndarray, C: np.ndarray) -> np.ndarray:
    """C - A B in K-word arithmetic (Sec. 2, Fig. 1: the library's block
    matrix multiplication): every entry takes its k multiply-subtracts in
    increasing k.  A (K, k, m), B (K, n, k), C (K, n, m), K-plane column-major
    (column index first); returns the new C."""
    A, B = _c(A), _c(B)
    C = _c(C).copy()
    _, k, m = A.shape
    n = B.shape[1]
    assert B.shape[2] == k and C.shape[1] == n and C.shape[2] == m
    lib().orc_gemm(K, m, n, k, _p(A), max(m, 1), max(m, 1) * k, _p(B), max(k, 1), max(k, 1) * n, _p(C), max(m, 1),
                   max(m, 1) * n)
    return C


def residual(A: np.ndarray, x: np.ndarray, b: np.ndarray) -> np.ndarray:
    """r = b - A x exactly, rounded to the canonical L-word form, L = the
    words of x and b (4: quad-double; 8: the 424-bit long precision)."""
    A, x, b = _c(A), _c(x), _c(b)
    aw, n, _ = A.shape
    lw = x.shape[0]
    assert lw in (4, 8) and x.shape == (lw, n) and b.shape == (lw, n)
    r = np.empty((lw, n))
    bad = lib().orc_residual(n, aw, lw, _p(A), n, n * n, _p(x), n, _p(b), n, _p(r), n)
    if bad:
        raise FloatingPointError("residual word outside the binary64 normal range")
    return r


def extend(v: np.ndarray, K: int = 4) -> np.ndarray:
    """Zero-extend a k-word vector to K words (exact)."""
    out = np.zeros((K, v.shape[1]))
    out[: v.shape[0]] = v
    return out


def norm2(v: np.ndarray) -> float:
    """2-norm of a binary64 vector, power-of-two scaled to avoid under/overflow."""
    v = np.abs(np.asarray(v, dtype=np.float64).ravel())
    m = float(v.max()) if v.size else 0.0
    if m == 0.0 or not math.isfinite(m):
        return m
    e = math.frexp(m)[1]
    s = np.ldexp(v, -e)
    return math.ldexp(math.sqrt(math.fsum((s * s).tolist())), e)


def refine(A: np.ndarray, b: np.ndarray, K: int, max_iter: int = 30,
           rtol: float = 0.0, atol: float = 0.0, ctol: float = 2.0 ** -208, ozaki: int = 0,
           escalate: bool = False, stag_ratio: float = 0.0, long_words: int = 4) -> dict:
    """Mixed-precision iterative refinement, Listing 1 of the paper (Sec. 2).

    A: (aw, n, n) with aw = 1 (binary64 entries) or 4 (quad-double entries).
    b: (m, n), m <= long_words words (zero-extended).  Factor precision K
    words; the long precision is L = long_words binary64 words, 4
    (quad-double) or 8 (424 bits, the long precision of the paper's Table
    2), with an exact residual rounded once to L words (the reading of the
    residual step); x and the update x + z are L-word.  Steps, in the
    listing's order:
      ||A||_F; K-word copies of A and b; LU + substitution; x to long;
      loop: r = b - A x; stop if ||r|| < sqrt(n) rtol ||A||_F ||x|| + atol
      (the listing's test, eq. (2)) or if the previous correction satisfied
      ||z||_inf <= ctol ||x||_inf (forward test added by this reading: the
      residual test certifies only a backward error, ~kappa * rtol forward);
      r <- r * 2^-e (power-of-two normalisation); K-word copy of r;
      substitution -> z; z <- 2^e z; x <- x + z.
    Norms are taken over leading words in binary64.  With ozaki = s > 0 the
    first factorisation is getrf_ozaki with s slices (panel width 64)
    instead of the plain LU.

    Stagnation (not in the paper; the escalation rule of this project):
    with stag_ratio > 0, once two corrections have been applied since the
    last factorisation, the loop checks after the convergence tests whether
    the last correction failed to shrink, ||z_i||_inf > stag_ratio *
    ||z_(i-1)||_inf.  Then, if escalate and K < 4, A is refactored in K+1
    words (plain LU) and the loop goes on from the current x; otherwise it
    stops with STAGNATED.  An exactly zero pivot escalates the same way.
    max_iter bounds the corrections over all precisions.  Returns a dict
    with x (4, n), iters (corrections applied), status, info, history of
    ||r||, final_words (K of the last factorisation), escalations, and the
    norms of the last test: resid_norm ||r||_2, x_norm ||x||_2 and a_norm
    ||A||_F (leading words).
    """
    A = _c(A)
    lw = long_words
    assert lw in (4, 8) and b.shape[0] <= lw
    b = extend(_c(b), lw)
    aw, n, _ = A.shape
    out = dict(x=np.zeros((lw, n)), iters=0, status=NONFINITE, info=0, history=[], final_words=K, escalations=0)
    if not (np.isfinite(A).all() and np.isfinite(b).all()):
        return out
    norm_a = norm2(A[0])
    out.update(a_norm=norm_a, resid_norm=0.0, x_norm=0.0)
    kc = K
    escalations = 0
    while True:
        LU = stage(kc, A)
        if ozaki and kc == K:
            LU0 = LU
            LU, ipiv, info = getrf_ozaki(kc, LU0, ozaki)
            if info == -3:  # the split scheme left its exact range: the plain form
                LU, ipiv, info = getrf(kc, LU0)
        else:
            LU, ipiv, info = getrf(kc, LU)
        if not info or not escalate or kc == 4:
            break
        kc += 1
        escalations += 1
    out.update(final_words=kc, escalations=escalations, info=info, LU=LU, ipiv=ipiv)
    if info:
        out.update(status=SINGULAR)
        return out
    x = extend(getrs(kc, LU, ipiv, round_words(kc, b)), lw)
    hist = []
    iters = 0
    status = MAX_ITER
    thresh_c = math.sqrt(n) * rtol * norm_a
    zs = []  # ||z||_inf of the corrections since the last factorisation
    for _ in range(max_iter + 1):
        r = residual(A, x, b)
        nr = norm2(r[0])
        nx = norm2(x[0])
        hist.append(nr)
        out.update(resid_norm=nr, x_norm=nx)
        xmax = float(np.abs(x[0]).max())
        if nr < thresh_c * nx + atol or (zs and zs[-1] <= ctol * xmax):
            status = CONVERGED
            break
        if stag_ratio > 0 and len(zs) >= 2 and zs[-1] > stag_ratio * zs[-2]:
            if not escalate or kc == 4:
                status = STAGNATED
                break
            while True:  # refactor in more words
                kc += 1
                escalations += 1
                LU, ipiv, info = getrf(kc, stage(kc, A))
                if not info or kc == 4:
                    break
            out.update(final_words=kc, escalations=escalations, info=info, LU=LU, ipiv=ipiv)
            if info:
                status = SINGULAR
                break
            zs = []
        if iters == max_iter:
            break
        e = math.frexp(float(np.abs(r[0]).max()))[1] - 1
        rf = round_words(kc, np.ldexp(r, -e))
        z = np.ldexp(extend(getrs(kc, LU, ipiv, rf), lw), e)
        zs.append(float(np.abs(z[0]).max()))
        x = add(lw, x, z)
        iters += 1
    out.update(x=x, iters=iters, status=status, history=hist)
    return out
