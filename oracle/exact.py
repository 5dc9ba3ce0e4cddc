"""ORACLE -- test infrastructure: exact rational definitions.

Plain ``fractions.Fraction`` versions of the quantities the solver
approximates, for pinning the C oracle on small inputs:
  * the exact value of a K-word number and its canonical rounding (greedy
    round-to-nearest: w0 = RN(v), w1 = RN(v - w0), ...);
  * LU with partial pivoting in exact arithmetic (Kouya 2021, Sec. 2: LU
    decomposition with partial pivoting; LAPACK getf2 conventions for the
    pivot choice: first row of largest magnitude, 0-based swap sequence);
  * the residual b - A x in exact arithmetic (Listing 1, residual step).
CPython's float(Fraction) divides two integers with correct rounding, so it
is an exact round-to-nearest-even of any rational.
"""
from __future__ import annotations

from fractions import Fraction
from typing import Sequence


def value(words: Sequence[float]) -> Fraction:
    """Exact value of an unevaluated sum of binary64 words."""
    s = Fraction(0)
    for w in words:
        s += Fraction(float(w))
    return s


def canon(q: Fraction, K: int) -> list[float]:
    """Canonical K-word rounding of a rational: greedy round-to-nearest."""
    out = []
    for _ in range(K):
        w = float(q)
        out.append(w)
        q = q - Fraction(w)
    return out


def lu_partial_pivot(A: list[list[Fraction]]):
    """Exact PA = LU with partial pivoting.  Returns (LU, ipiv, info) where
    LU holds L (unit, strictly lower) and U in place, ipiv the 0-based swap
    sequence, info 0 or k+1 at the first zero pivot."""
    n = len(A)
    a = [list(map(Fraction, row)) for row in A]
    ipiv = [0] * n
    info = 0
    for k in range(n):
        p = k
        for i in range(k + 1, n):
            if abs(a[i][k]) > abs(a[p][k]):
                p = i
        ipiv[k] = p
        a[k], a[p] = a[p], a[k]
        if a[k][k] == 0:
            if info == 0:
                info = k + 1
            continue
        for i in range(k + 1, n):
            a[i][k] = a[i][k] / a[k][k]
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                a[i][j] -= a[i][k] * a[k][j]
    return a, ipiv, info


def pivot_gaps(A: list[list[Fraction]]) -> list[Fraction]:
    """Relative gap between the chosen pivot and the runner-up at each step
    of exact partial pivoting: (|a_pk| - max_{i != p} |a_ik|) / |a_pk|.
    A step whose gap is tiny is a near-tie that finite precision may break
    differently."""
    n = len(A)
    a = [list(map(Fraction, row)) for row in A]
    gaps = []
    for k in range(n):
        mags = [abs(a[i][k]) for i in range(k, n)]
        p = k + max(range(len(mags)), key=lambda t: (mags[t], -t))
        best = mags[p - k]
        rest = [m for t, m in enumerate(mags) if t != p - k]
        gaps.append(Fraction(1) if best == 0 or not rest else (best - max(rest)) / best)
        a[k], a[p] = a[p], a[k]
        if a[k][k] == 0:
            continue
        for i in range(k + 1, n):
            a[i][k] = a[i][k] / a[k][k]
        for i in range(k + 1, n):
            for j in range(k + 1, n):
                a[i][j] -= a[i][k] * a[k][j]
    return gaps


def residual(A_words, x_words, b_words) -> list[Fraction]:
    """Exact b - A x.  A_words[i][j] is a sequence of words of entry (i, j);
    x_words[j], b_words[i] sequences of words."""
    n = len(b_words)
    xs = [value(x) for x in x_words]
    out = []
    for i in range(n):
        s = value(b_words[i])
        for j in range(n):
            s -= value(A_words[i][j]) * xs[j]
        out.append(s)
    return out
