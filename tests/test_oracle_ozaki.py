"""Pins for the oracle's split form of the trailing update (error-free
splitting after Ozaki, Ogita, Oishi and Rump, Numer. Algorithms 59 (2012)),
the project's alternative to the K-word trailing update of the paper's LU
(Kouya 2021, Sec. 2).

What the mathematics fixes, checked here with exact rationals:
  * the slices of a value plus its remainder equal the value exactly, each
    slice is a multiple of its grid and within the stated magnitude bound;
  * every group sum acc_d is exactly the rational sum of its slice products;
  * C - L U computed this way is within the truncation + rounding bound of
    the exact C - L U;
  * on matrices whose exact factors are short dyadics the split LU returns
    those factors bit for bit, for every K and slice count;
  * refinement on top of the split factor reaches the quad-double solution.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import synth
from helpers import rand_words
from oracle import exact as X

def F(v):
    return Fraction(float(v))


def slice_bound(K, q, beta):
    """|slice_q| / grid_q <= this (see the scheme's exactness argument)."""
    return Fraction(2) ** beta + Fraction(K, 2) if q == 0 else K * Fraction(2) ** (beta - 1) + Fraction(K, 2)


def group_bound(K, s, beta, kb=64):
    """Largest possible |acc_d| over d < s, in units of the group's grid."""
    b = [slice_bound(K, q, beta) for q in range(s)]
    return max(kb * sum(b[p] * b[d - p] for p in range(d + 1)) for d in range(s))


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_slice_width_is_the_widest_exact_one(K):
    """beta(K, s) keeps every group sum of a depth-64 update below 2^53
    grid units and one more bit would not; the widths the forms use: 22 for
    a double-double factor with 5 slices (110 bits, above its 106), 21 for
    triple-double with 5, 20 for quad-double with 11 and for 16 slices of
    triple- or quad-double."""
    for s in range(1, O.OZ_SMAX + 1):
        beta = O.oz_beta(K, s)
        assert group_bound(K, s, beta) < Fraction(2) ** 53
        assert beta == 26 or group_bound(K, s, beta + 1) >= Fraction(2) ** 53
        if s > 1:
            assert beta <= O.oz_beta(K, s - 1)
    assert O.oz_beta(2, 5) == 22 and O.oz_beta(3, 5) == 21 and O.oz_beta(4, 11) == 20
    assert O.oz_beta(3, 16) == O.oz_beta(4, 16) == 20
    with pytest.raises(ValueError):
        O.oz_beta(K, 0)
    with pytest.raises(ValueError):
        O.oz_beta(K, O.OZ_SMAX + 1)


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_slices_sum_exactly_and_sit_on_their_grids(K):
    g = np.random.default_rng(700 + K)
    for trial in range(12):
        m = 24
        x = rand_words(g, K, m, spread=30)
        E = O.oz_scale(x[0])
        top = max(abs(v) for v in x[0])
        assert top < 2.0 ** E and top >= 2.0 ** (E - 1)
        for s in (1, 3, 5, 8, 16):
            sl, rem = O.oz_slices(K, s, x, E)
            beta = O.oz_beta(K, s)
            for i in range(m):
                total = sum((F(v) for v in sl[:, i]), Fraction(0)) + X.value(rem[:, i])
                assert total == X.value(x[:, i])
                for q in range(s):
                    grid = Fraction(2) ** (E - (q + 1) * beta)
                    units = F(sl[q, i]) / grid
                    assert units.denominator == 1
                    assert abs(units) <= slice_bound(K, q, beta)
                # what is left is below half a grid step per word
                assert abs(X.value(rem[:, i])) <= K * Fraction(2) ** (E - s * beta) / 2
            if s == 16:  # 320 bits below the top reach every word's last bit
                assert np.all(rem == 0.0)


def test_scale_of_zero_and_powers_of_two():
    assert O.oz_scale(np.zeros(5)) == 0
    assert O.oz_scale(np.array([0.0, 1.0, -0.5])) == 1   # |x| < 2^1
    assert O.oz_scale(np.array([-0.75])) == 0
    assert O.oz_scale(np.array([3.0 * 2.0 ** -600])) == -598


def blocks(g, K, m, kb, nc, spread):
    L = np.zeros((K, kb, m))
    U = np.zeros((K, nc, kb))
    C = np.zeros((K, nc, m))
    for k in range(kb):
        L[:, k, :] = rand_words(g, K, m, spread)
    for j in range(nc):
        U[:, j, :] = rand_words(g, K, kb, spread)
        C[:, j, :] = rand_words(g, K, m, spread)
    return L, U, C


@pytest.mark.parametrize("K,s", [(2, 16), (3, 16), (4, 16), (2, 5), (2, 7), (3, 5), (4, 11), (1, 3)])
def test_group_sums_are_exact_at_full_width(K, s):
    """kb = 64: the largest group has 64 * s products; with every entry near
    the top of its binade and the lower words near half a step of the grid
    the sums come closest to the bound.  Each acc_d must equal the rational
    sum exactly, at the widest slices beta(K, s) allows."""
    g = np.random.default_rng(720 + K + 31 * s)
    m, kb, nc = 3, 64, 2
    beta = O.oz_beta(K, s)
    L, U, C = blocks(g, K, m, kb, nc, spread=0)
    # push every leading word to the top of [1/2, 1), signs aligned so that
    # the group sums add up instead of cancelling
    L[0] = 1.0 - 2.0 ** -53
    U[0] = 1.0 - 2.0 ** -53
    _, acc = O.oz_update(K, s, L, U, C)
    largest = Fraction(0)
    for i in range(m):
        E = O.oz_scale(L[0, :, i])
        Ls, _ = O.oz_slices(K, s, L[:, :, i], E)
        for j in range(nc):
            Fc = O.oz_scale(U[0, j, :])
            Us, _ = O.oz_slices(K, s, U[:, j, :], Fc)
            for d in range(s):
                exact = sum((F(Ls[p, k]) * F(Us[d - p, k]) for p in range(d + 1) for k in range(kb)), Fraction(0))
                assert F(acc[d, j, i]) == exact, (i, j, d)
                grid = Fraction(2) ** (E + Fc - (d + 2) * beta)
                assert (exact / grid).denominator == 1
                assert abs(exact / grid) < Fraction(2) ** 53
                largest = max(largest, abs(exact / grid))
    # the test reaches the bound's order of magnitude (within a factor 16)
    assert largest * 16 > group_bound(K, s, beta) / (s if s > 1 else 1)


@pytest.mark.parametrize("K", [2, 3, 4])
@pytest.mark.parametrize("s", [2, 5, 8, 12])
def test_update_within_truncation_and_rounding_bound(K, s):
    g = np.random.default_rng(740 + 10 * K + s)
    m, kb, nc = 5, 13, 4
    L, U, C = blocks(g, K, m, kb, nc, spread=4)
    Cn, acc = O.oz_update(K, s, L, U, C)
    uK = Fraction(2) ** (-53 * K)
    for i in range(m):
        E = O.oz_scale(L[0, :, i])
        for j in range(nc):
            Fc = O.oz_scale(U[0, j, :])
            lu = sum((X.value(L[:, k, i]) * X.value(U[:, j, k]) for k in range(kb)), Fraction(0))
            exact = X.value(C[:, j, i]) - lu
            got = X.value(Cn[:, j, i])
            beta = O.oz_beta(K, s)
            trunc = kb * Fraction(2) ** (E + Fc - s * beta) * (Fraction(41, 10) * (s + 1) + K + 1)
            comb = 8 * s * uK * (abs(X.value(C[:, j, i])) + sum(abs(F(a)) for a in acc[:, j, i]))
            assert abs(got - exact) <= trunc + comb, (i, j)


def test_update_pairs_each_row_slice_with_the_right_column_slice():
    """A planted pairing mistake (L_p with U_p instead of U_{d-p}) would move
    the result by about 2^-20 relative; the bound above is far tighter."""
    g = np.random.default_rng(777)
    K, s = 3, 6
    L, U, C = blocks(g, K, 4, 9, 3, spread=0)
    Cn, acc = O.oz_update(K, s, L, U, C)
    i, j = 1, 2
    lu = sum((X.value(L[:, k, i]) * X.value(U[:, j, k]) for k in range(9)), Fraction(0))
    assert abs(sum(F(a) for a in acc[:, j, i]) - lu) <= abs(lu) * Fraction(2) ** -100 + Fraction(2) ** -100


def to_planes(A, K):
    P = np.zeros((K, A.shape[0], A.shape[0]))
    P[0] = A.T
    return P


def constructed(n, g):
    L = np.tril(g.integers(-7, 8, (n, n)) / 8.0, -1) + np.eye(n)
    U = np.triu(g.integers(-9, 10, (n, n)).astype(float), 1)
    U += np.diag(g.choice([-4.0, -2.0, -1.0, 1.0, 2.0, 4.0], n))
    perm = g.permutation(n)
    return (L @ U)[np.argsort(perm)], L, U


@pytest.mark.parametrize("K", [1, 2, 3, 4])
@pytest.mark.parametrize("nb,s", [(4, 2), (7, 8), (16, 16), (64, 3)])
def test_constructed_factorisation_exact(K, nb, s):
    g = np.random.default_rng(800 + K + nb)
    for n in (1, 5, 33, 70):
        A, L, U = constructed(n, g)
        assert np.abs(A).max() < 2.0 ** 40
        LU, ipiv, info = O.getrf_ozaki(K, to_planes(A, K), s, nb)
        LUp, ipp, _ = O.getrf(K, to_planes(A, K))
        assert info == 0
        np.testing.assert_array_equal(ipiv, ipp)
        M = LU[0].T
        np.testing.assert_array_equal(np.tril(M, -1) + np.eye(n), L)
        np.testing.assert_array_equal(np.triu(M), U)
        assert np.all(LU[1:] == 0.0)


def test_bad_parameters_rejected():
    A = to_planes(np.eye(3), 2)
    with pytest.raises(ValueError):
        O.getrf_ozaki(2, A, 0)
    with pytest.raises(ValueError):
        O.getrf_ozaki(2, A, 17)
    with pytest.raises(ValueError):
        O.getrf_ozaki(2, A, 4, nb=65)


def test_singular_info_matches_plain_lu():
    A = np.array([[1.0, 2.0, 3.0, 1.0], [2.0, 4.0, 6.0, 2.0], [1.0, 0.0, 1.0, 5.0], [0.0, 1.0, 1.0, 1.0]])
    for K in (2, 3):
        _, _, info = O.getrf_ozaki(K, to_planes(A, K), 4, nb=2)
        _, _, info_p = O.getrf(K, to_planes(A, K))
        assert info == info_p != 0


@pytest.mark.parametrize("K,s,cond", [(2, 4, 1e8), (3, 6, 1e10), (4, 9, 1e15), (3, 2, 1e3)])
def test_refinement_on_split_factor_reaches_quad_double(K, s, cond):
    """The split factor is a little less accurate than the plain K-word one;
    the refinement loop must still end at the quad-double solution (exact
    solution all ones, right-hand side exact in quad-double)."""
    Ap, b, exact = synth.problem("randsvd", 130, config=1, instance=40 + s, cond=cond)
    assert exact
    r = O.refine(Ap, b, K, ozaki=s)
    assert r["status"] == O.CONVERGED
    err = max(abs(X.value(r["x"][:, i]) - 1) for i in range(130))
    assert err <= Fraction(10) ** -60


# ---- the exact range of the scheme ------------------------------------------

@pytest.mark.parametrize("K,s", [(1, 3), (2, 4), (2, 5), (3, 7), (4, 11), (4, 16)])
def test_exact_range_bound_is_the_tightest_symmetric_one(K, s):
    """oz_emin(K, s) is the smallest scale E such that two scales at E keep
    every slice grid 2^(E - (q+1) beta), q < s, and every kept product grid
    2^(E + F - (d+2) beta), d < s, at 2^-1022 or above; one below it does
    not.  Written out from the grids, not from the closed form."""
    b = O.oz_beta(K, s)
    e = O.oz_emin(K, s)

    def normal(E, F):
        return (all(E - (q + 1) * b >= -1022 and F - (q + 1) * b >= -1022 for q in range(s))
                and all(E + F - (d + 2) * b >= -1022 for d in range(s)))
    assert normal(e, e)
    assert not normal(e - 1, e - 1)
    assert normal(e, 0) and normal(0, e)  # one side larger only helps


@pytest.mark.parametrize("K,s", [(2, 4), (3, 5), (4, 11)])
def test_group_sums_are_exact_at_the_range_bound(K, s):
    """Rows and columns scaled (by exact powers of two) to scale oz_emin:
    every group sum is still the rational sum of its slice products."""
    g = np.random.default_rng(940 + K + 17 * s)
    m, kb, nc = 2, 64, 2
    e = O.oz_emin(K, s)
    L, U, C = blocks(g, K, m, kb, nc, spread=0)
    L[0] = 1.0 - 2.0 ** -53
    U[0] = 1.0 - 2.0 ** -53
    L, U = np.ldexp(L, e), np.ldexp(U, e)
    _, acc = O.oz_update(K, s, L, U, C)
    for i in range(m):
        E = O.oz_scale(L[0, :, i])
        assert E == e
        Ls, _ = O.oz_slices(K, s, L[:, :, i], E)
        for j in range(nc):
            Fc = O.oz_scale(U[0, j, :])
            Us, _ = O.oz_slices(K, s, U[:, j, :], Fc)
            for d in range(s):
                exact = sum((F(Ls[p, k]) * F(Us[d - p, k]) for p in range(d + 1) for k in range(kb)), Fraction(0))
                assert F(acc[d, j, i]) == exact, (i, j, d)


def test_factorisation_below_the_range_reports_it_and_refinement_uses_the_plain_form():
    """A matrix scaled well below the range (its U12 columns' scales under
    oz_emin; U12 = L11^-1 A12 may grow a few bits over A) makes the split LU
    report info = -3; the refinement then factors in the plain form, so its
    result is the plain refinement's.  Scaled well above, nothing is
    reported."""
    K, s, n = 2, 4, 100
    Ap, b, exact = synth.problem("uniform", n, config=1, instance=77)
    assert exact
    e = O.oz_emin(K, s)
    low, ok = np.ldexp(Ap, e - 20), np.ldexp(Ap, e + 20)
    _, _, info = O.getrf_ozaki(K, O.stage(K, low), s)
    assert info == -3
    _, _, info = O.getrf_ozaki(K, O.stage(K, ok), s)
    assert info == 0
    bl = np.ldexp(b, e - 20)
    r = O.refine(low, bl, K, ozaki=s)
    p = O.refine(low, bl, K)
    assert r["status"] == p["status"] == O.CONVERGED and r["iters"] == p["iters"]
    np.testing.assert_array_equal(r["x"], p["x"])
