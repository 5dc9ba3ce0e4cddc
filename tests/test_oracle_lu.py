"""Pins for the oracle's LU with partial pivoting and the substitutions
(Kouya 2021, Sec. 2: LU decomposition with partial pivoting and
forward/backward substitution in DD/TD/QD arithmetic).

Independent references: LAPACK (scipy.linalg.lu_factor / lu_solve) for the
binary64 case, exact rational LU for tiny matrices, and matrices built as
P^T L U from dyadic factors whose every intermediate value is exactly
representable, so that every precision must reproduce L, U and the pivots
bit for bit.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
from oracle import exact as X


def to_planes(A, K=1):
    P = np.zeros((K, A.shape[0], A.shape[0]))
    P[0] = A.T
    return P


def unpack(LU, n):
    """(L, U) as binary64 leading-word dense matrices from a K-plane LU."""
    M = LU[0].T
    return np.tril(M, -1) + np.eye(n), np.triu(M)


def apply_swaps(A, ipiv):
    A = A.copy()
    for k, p in enumerate(ipiv):
        if p != k:
            A[[k, p]] = A[[p, k]]
    return A


@pytest.mark.parametrize("n", [17, 64, 200])
def test_k1_matches_lapack(n):
    g = np.random.default_rng(n)
    A = g.uniform(-1, 1, (n, n))
    LU, ipiv, info = O.getrf(1, to_planes(A))
    lu, piv = sla.lu_factor(A)
    assert info == 0
    np.testing.assert_array_equal(ipiv, piv)
    np.testing.assert_allclose(LU[0].T, lu, rtol=0, atol=1e-11 * np.abs(lu).max())
    b = g.uniform(-1, 1, n)
    x = O.getrs(1, LU, ipiv, b[None, :])[0]
    np.testing.assert_allclose(x, sla.lu_solve((lu, piv), b), rtol=1e-9, atol=1e-9)


def constructed(n, g, K):
    """A = P^T L U with L unit lower (entries j/8, |l| < 1), U upper with
    small-integer off-diagonal and power-of-two diagonal entries."""
    L = np.tril(g.integers(-7, 8, (n, n)) / 8.0, -1) + np.eye(n)
    U = np.triu(g.integers(-9, 10, (n, n)).astype(float), 1)
    U += np.diag(g.choice([-4.0, -2.0, -1.0, 1.0, 2.0, 4.0], n))
    perm = g.permutation(n)
    A = (L @ U)[np.argsort(perm)]  # row perm[i] of A is row i of L U
    return A, L, U


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_constructed_factorisation_exact(K):
    g = np.random.default_rng(40 + K)
    for n in (1, 2, 5, 16, 33):
        A, L, U = constructed(n, g, K)
        assert np.abs(A).max() < 2.0 ** 40  # every partial sum is an exact dyadic
        LU, ipiv, info = O.getrf(K, to_planes(A, K))
        assert info == 0
        Lg, Ug = unpack(LU, n)
        np.testing.assert_array_equal(Lg, L)
        np.testing.assert_array_equal(Ug, U)
        assert np.all(LU[1:] == 0.0)
        np.testing.assert_array_equal(apply_swaps(A, ipiv), L @ U)
        # exact known solution
        x = g.integers(-5, 6, n).astype(float)
        b = A @ x
        xs = O.getrs(K, LU, ipiv, np.vstack([b, np.zeros((K - 1, n))]))
        np.testing.assert_array_equal(xs[0], x)
        assert np.all(xs[1:] == 0.0)


def random_int_matrix_without_near_ties(g, n):
    while True:
        A = g.integers(-20, 21, (n, n)).astype(float)
        gaps = X.pivot_gaps(A.tolist())
        if min(gaps) > Fraction(1, 1000) and abs(np.linalg.det(A)) > 0.5:
            return A


@pytest.mark.parametrize("K", [2, 3, 4])
def test_small_against_exact_rational_lu(K):
    g = np.random.default_rng(60 + K)
    u = Fraction(2) ** (-53 * K)
    for n in (3, 6, 9):
        for _ in range(4):
            A = random_int_matrix_without_near_ties(g, n)
            LUx, ipx, infox = X.lu_partial_pivot(A.tolist())
            LU, ipiv, info = O.getrf(K, to_planes(A, K))
            assert info == infox == 0
            assert list(ipiv) == ipx
            scale = max(abs(v) for row in LUx for v in row)
            for i in range(n):
                for j in range(n):
                    got = X.value(LU[:, j, i])
                    assert abs(got - LUx[i][j]) <= 64 * n * u * scale


def test_singular_info():
    A = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [1.0, 0.0, 1.0]])
    for K in (1, 2, 3, 4):
        _, _, info = O.getrf(K, to_planes(A, K))
        assert info == 3  # exact zero pivot at the last step
    Z = np.zeros((4, 4))
    Z[:, 1:] = np.random.default_rng(0).uniform(-1, 1, (4, 3))
    _, ipiv, info = O.getrf(3, to_planes(Z, 3))
    assert info == 1 and ipiv[0] == 0


def test_ties_take_first_row():
    """Equal magnitudes: the first row (smallest index) is the pivot, as in
    LAPACK's i?amax."""
    A = np.array([[1.0, 1.0, 0.0], [-2.0, 0.5, 1.0], [2.0, 3.0, 1.0]])
    for K in (1, 2, 3, 4):
        _, ipiv, _ = O.getrf(K, to_planes(A, K))
        assert ipiv[0] == 1
    _, piv = sla.lu_factor(A)
    assert piv[0] == 1


@pytest.mark.parametrize("K", [2, 3, 4])
def test_known_solution_forward_error(K):
    """getrf + getrs on A x = A*ones (exact rhs): forward error within the
    usual n * kappa * u_K bound (Kouya 2021 Table 1 shows the same
    precision ladder)."""
    import synth
    n = 48
    Ap, b, exact = synth.problem("uniform", n, config=0, instance=7)
    assert exact
    kappa = np.linalg.cond(Ap[0].T, 1)
    LU, ipiv, info = O.getrf(K, O.stage(K, Ap))
    x = O.getrs(K, LU, ipiv, O.round_words(K, b))
    err = max(abs(X.value(x[:, i]) - 1) for i in range(n))
    assert err <= 10 * n * kappa * 2.0 ** (-53 * K)
