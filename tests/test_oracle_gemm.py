"""Pins for the oracle's multi-word matrix multiply-subtract C - A B (the
block matrix multiplication of the multi-word library the paper's direct
methods are built on, Kouya 2021, Sec. 2 and Fig. 1), every entry taking
its k multiply-subtracts in increasing k.

What the mathematics fixes, checked here:
  * with operands whose products and partial sums are exact in K words
    (small integers, short dyadics) the result is the exact C - A B, bit for
    bit, for every K; non-square shapes with distinct entries make a
    transposed or misindexed operand fail;
  * on general multi-word inputs the error stays within the accumulated
    multiply-subtract bound of the word arithmetic against exact rationals;
  * k = 0 leaves C as it was.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from helpers import rand_words
from oracle import exact as X


def planes(M, K):
    """K-plane column-major storage of a binary64 matrix M (rows x cols)."""
    P = np.zeros((K, M.shape[1], M.shape[0]))
    P[0] = M.T
    return P


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_small_integers_exact(K):
    g = np.random.default_rng(60 + K)
    m, n, k = 7, 5, 9
    A = g.integers(-40, 41, (m, k)).astype(float)
    B = g.integers(-40, 41, (k, n)).astype(float)
    C = g.integers(-1000, 1001, (m, n)).astype(float)
    R = O.gemm(K, planes(A, K), planes(B, K), planes(C, K))
    np.testing.assert_array_equal(R[0].T, C - A @ B)
    assert np.all(R[1:] == 0.0)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_short_dyadics_exact_in_k_words(K):
    """Entries of 20 significant bits spread over 17 binades: the exact
    value of every partial sum spans at most ~80 bits (products of 40 bits
    spread over 32 binades, a few bits of carries), beyond one word but
    within two, so every K-word multiply-subtract is exact."""
    g = np.random.default_rng(80 + K)
    m, n, k = 6, 4, 11
    A = g.integers(-2 ** 19, 2 ** 19, (m, k)) * np.exp2(g.integers(-8, 9, (m, k)))
    B = g.integers(-2 ** 19, 2 ** 19, (k, n)) * np.exp2(g.integers(-8, 9, (k, n)))
    C = g.integers(-2 ** 19, 2 ** 19, (m, n)) * np.exp2(g.integers(-16, 17, (m, n)))
    R = O.gemm(K, planes(A, K), planes(B, K), planes(C, K))
    for i in range(m):
        for j in range(n):
            exact = Fraction(C[i, j]) - sum((Fraction(A[i, l]) * Fraction(B[l, j]) for l in range(k)), Fraction(0))
            assert X.value(R[:, j, i]) == exact, (i, j)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_general_words_within_bound(K):
    """|C - A B computed - exact| <= sum over the k steps of the
    multiply-subtract bound 8 u_K (|c| + |a b|), u_K = 2^(-53K), with |c|
    bounded by |C| + the sum of |a b| so far."""
    g = np.random.default_rng(90 + K)
    m, n, k = 5, 3, 8
    A = np.stack([rand_words(g, K, m, spread=6) for _ in range(k)], axis=1)   # (K, k, m)
    B = np.stack([rand_words(g, K, k, spread=6) for _ in range(n)], axis=1)   # (K, n, k)
    C = np.stack([rand_words(g, K, m, spread=6) for _ in range(n)], axis=1)   # (K, n, m)
    R = O.gemm(K, A, B, C)
    u = Fraction(2) ** (-53 * K)
    for i in range(m):
        for j in range(n):
            c0 = X.value(C[:, j, i])
            prods = [X.value(A[:, l, i]) * X.value(B[:, j, l]) for l in range(k)]
            exact = c0 - sum(prods, Fraction(0))
            run, bound = abs(c0), Fraction(0)
            for p in prods:
                bound += 8 * u * (run + abs(p))
                run += abs(p) + 8 * u * (run + abs(p))
            assert abs(X.value(R[:, j, i]) - exact) <= bound, (i, j)
            # a dropped last term would be off by |p_last|, far above the bound
            assert abs(prods[-1]) > 1000 * bound


def test_empty_inner_dimension_leaves_c():
    g = np.random.default_rng(3)
    C = rand_words(g, 3, 12).reshape(3, 3, 4)
    R = O.gemm(3, np.zeros((3, 0, 4)), np.zeros((3, 3, 0)), C)
    np.testing.assert_array_equal(R, C)
