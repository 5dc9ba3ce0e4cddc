"""The multi-word randsvd generator (entries kept in up to four binary64
words for condition numbers binary64 entries cannot carry) against exact
rational arithmetic: the stored entries equal U diag(sigma) V^T (the same
seeded U, V, sigma) to about 150 bits of each row's scale, the words of an
entry do not overlap, and the right-hand side b = A * ones is exact."""
from fractions import Fraction

import numpy as np

import synth


def test_randsvd_words_matches_exact_product():
    n, cond = 40, 1e25
    Ap = synth.randsvd_words(n, cond, synth.rng(11, 0))
    g = synth.rng(11, 0)
    U = synth.haar(n, g)
    V = synth.haar(n, g)
    sig = cond ** (-np.arange(n) / (n - 1))
    for i in range(0, n, 3):
        row_scale = float(np.abs(U[i] * sig).max() * np.abs(V).max())
        for j in range(0, n, 4):
            exact = sum((Fraction(float(U[i, k])) * Fraction(float(sig[k])) * Fraction(float(V[j, k]))
                         for k in range(n)), Fraction(0))
            stored = sum((Fraction(float(Ap[w, j, i])) for w in range(4)), Fraction(0))
            assert abs(float(exact - stored)) <= 2.0 ** -140 * row_scale, (i, j)


def test_randsvd_words_are_nonoverlapping_and_rhs_exact():
    n = 64
    Ap, b, exact = synth.problem("randsvd_words", n, config=11, instance=1, cond=1e30)
    assert Ap.shape == (4, n, n) and exact
    w0, w1, w2 = np.abs(Ap[0]), np.abs(Ap[1]), np.abs(Ap[2])
    # each word below half an ulp of the one before it (or zero)
    assert np.all((w1 == 0) | (w1 <= np.spacing(w0) / 2 * (1 + 1e-15)))
    assert np.all((w2 == 0) | (w2 <= np.spacing(w1) / 2 * (1 + 1e-15)))
    # b = A * ones exactly: the words of b hold every row sum
    for i in range(0, n, 7):
        s = sum((Fraction(float(Ap[w, j, i])) for w in range(4) for j in range(n)), Fraction(0))
        assert s == sum((Fraction(float(v)) for v in b[:, i]), Fraction(0))


def test_randsvd_words_keeps_the_condition_number():
    """Binary64 entries cap a matrix labelled 1e30 near 1e16-1e18; the word
    entries keep it: the smallest singular value of the stored matrix,
    computed from the exact entries in high precision, is near 1e-30."""
    import mpmath
    n = 24
    Ap = synth.randsvd_words(n, 1e30, synth.rng(11, 2))
    mpmath.mp.prec = 400
    M = mpmath.matrix(n, n)
    for i in range(n):
        for j in range(n):
            M[i, j] = sum(mpmath.mpf(float(Ap[w, j, i])) for w in range(4))
    s = mpmath.svd_r(M, compute_uv=False)
    smin = min(abs(v) for v in s)
    smax = max(abs(v) for v in s)
    assert 0.5e30 < smax / smin < 2e30


def test_paper_problem_condition_number_and_exact_rhs():
    """The paper's system (Sec. 3): A = R D R^-1 with d_i = 10^(-26 (i-1)/n)
    has kappa_2(A) = 10^(26 (n-1)/n) (R orthogonal here), and b = A x for
    x = [0, 1, ..., n-1] holds exactly in the four words of b; A is
    symmetric up to its entries' row grids (~2^-150 of the row scale)."""
    import mpmath
    n = 24
    Ap, b, exact, xs = synth.paper_problem(n, instance=1)
    assert exact
    np.testing.assert_array_equal(xs, np.arange(n))
    for i in range(n):
        s = sum((Fraction(float(Ap[w, j, i])) * int(xs[j]) for w in range(4) for j in range(n)), Fraction(0))
        assert s == sum((Fraction(float(v)) for v in b[:, i]), Fraction(0))
    mpmath.mp.prec = 400
    M = mpmath.matrix(n, n)
    for i in range(n):
        for j in range(n):
            M[i, j] = sum(mpmath.mpf(float(Ap[w, j, i])) for w in range(4))
    amax = max(abs(M[i, j]) for i in range(n) for j in range(n))
    assert max(abs(M[i, j] - M[j, i]) for i in range(n) for j in range(n)) <= amax * mpmath.mpf(2) ** -140
    s = mpmath.svd_r(M, compute_uv=False)
    ratio = max(abs(v) for v in s) / min(abs(v) for v in s)
    want = mpmath.mpf(10) ** (mpmath.mpf(26) * (n - 1) / n)
    assert abs(ratio / want - 1) < 0.01
