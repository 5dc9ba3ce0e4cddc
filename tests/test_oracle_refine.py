"""Pins for the oracle's exact residual and its iterative-refinement loop
(Kouya 2021, Sec. 2, Listing 1; stopping rule eq. (2) of Sec. 3).

The residual is checked bit for bit against Fraction arithmetic rounded
greedily to quad-double.  The refinement is checked against systems whose
exact solution is known (b = A * ones formed exactly), against the
listing's step order (max_iter = 0, 1), and against its failure cases.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import synth
from oracle import exact as X


def rand_qd_vec(g, n, scale=1.0):
    out = np.zeros((4, n))
    for i in range(n):
        q = Fraction(0)
        for w in range(6):
            q += Fraction(float(g.uniform(-1, 1))) * Fraction(2) ** (-53 * w)
        out[:, i] = X.canon(q * Fraction(scale), 4)
    return out


@pytest.mark.parametrize("aw", [1, 4])
def test_residual_bitexact_vs_fraction(aw):
    g = np.random.default_rng(7 + aw)
    for n in (1, 3, 8):
        A = np.zeros((aw, n, n))
        for i in range(n):
            for j in range(n):
                q = sum((Fraction(float(g.uniform(-1, 1))) * Fraction(2) ** (-53 * w) for w in range(aw + 1)),
                        Fraction(0))
                A[:, j, i] = X.canon(q, aw)
        x = rand_qd_vec(g, n)
        b = rand_qd_vec(g, n, scale=2.0 ** int(g.integers(-3, 4)))
        r = O.residual(A, x, b)
        ex = X.residual([[A[:, j, i] for j in range(n)] for i in range(n)],
                        [x[:, j] for j in range(n)], [b[:, i] for i in range(n)])
        for i in range(n):
            assert list(r[:, i]) == X.canon(ex[i], 4)


def test_residual_zero_at_exact_solution():
    Ap, b, exact = synth.problem("uniform", 40, config=0, instance=3)
    assert exact
    x = np.zeros((4, 40))
    x[0] = 1.0
    np.testing.assert_array_equal(O.residual(Ap, x, b), 0.0)


def max_rel_err_vs_ones(x):
    return max(float(abs(X.value(x[:, i]) - 1)) for i in range(x.shape[1]))


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_refine_uniform_reaches_qd_accuracy(K):
    n = 64
    Ap, b, exact = synth.problem("uniform", n, config=0, instance=1)
    assert exact
    res = O.refine(Ap, b, K)
    assert res["status"] == O.CONVERGED
    assert max_rel_err_vs_ones(res["x"]) <= 1e-60
    # each correction gains at least ~a factor kappa*u_K: more words, fewer steps
    assert res["iters"] <= {1: 8, 2: 5, 3: 4, 4: 3}[K]


@pytest.mark.parametrize("K,cond", [(2, 1e10), (3, 1e10), (2, 1e15), (3, 1e15)])
def test_refine_randsvd_reaches_qd_accuracy(K, cond):
    n = 64
    Ap, b, exact = synth.problem("randsvd", n, config=2, instance=0, cond=cond)
    assert exact
    res = O.refine(Ap, b, K)
    assert res["status"] == O.CONVERGED
    assert max_rel_err_vs_ones(res["x"]) <= 1e-60
    # residual norms decrease until x reaches its quad-double rounding
    h = res["history"]
    assert all(h[i + 1] < h[i] for i in range(len(h) - 2))


def test_paper_residual_test_alone_stops_at_kappa_times_rtol():
    """With only eq. (2) (rtol near the quad-double unit roundoff) the loop
    stops once the backward error is small; the forward error is then
    limited by kappa * rtol, which is why the forward test is added."""
    n = 64
    Ap, b, _ = synth.problem("randsvd", n, config=2, instance=0, cond=1e15)
    res = O.refine(Ap, b, 2, rtol=2.0 ** -209, ctol=0.0)
    assert res["status"] == O.CONVERGED
    err = max_rel_err_vs_ones(res["x"])
    assert err <= 1e15 * 2.0 ** -209 * np.sqrt(n) * 100


def test_refine_step_order():
    """max_iter = 0 returns the unrefined short-precision solution; one
    correction equals solve + getrs(residual) + update done by hand."""
    n = 32
    K = 2
    Ap, b, _ = synth.problem("uniform", n, config=0, instance=5)
    r0 = O.refine(Ap, b, K, max_iter=0)
    LU, ipiv, info = O.getrf(K, O.stage(K, Ap))
    x0 = O.extend(O.getrs(K, LU, ipiv, O.round_words(K, b)))
    np.testing.assert_array_equal(r0["x"], x0)
    assert r0["iters"] == 0 and r0["status"] == O.MAX_ITER
    r1 = O.refine(Ap, b, K, max_iter=1)
    r = O.residual(Ap, x0, b)
    e = np.frexp(np.abs(r[0]).max())[1] - 1
    z = O.getrs(K, LU, ipiv, O.round_words(K, np.ldexp(r, -e)))
    x1 = O.add(4, x0, np.ldexp(O.extend(z), e))
    np.testing.assert_array_equal(r1["x"], x1)
    assert r1["iters"] == 1


def test_refine_failure_modes():
    # rows 1 and 3 of an integer matrix are equal: elimination is exact and
    # meets an exactly zero pivot
    A = np.array([[2.0, 1, 0, 1], [1, 3, 1, 0], [0, 1, 4, 1], [1, 3, 1, 0]])
    Ap = synth.planes(A)
    b, _ = synth.rhs_ones(Ap)
    assert O.refine(Ap, b, 3)["status"] == O.SINGULAR
    Ap2 = Ap.copy()
    Ap2[0, 2, 2] = np.nan
    assert O.refine(Ap2, b, 3)["status"] == O.NONFINITE


# ---------------------------------------------------------------------------
# stagnation and escalation (the project's rule on top of Listing 1)
# ---------------------------------------------------------------------------

def _err_vs_ones(x):
    from oracle import exact as X
    return max(abs(X.value(x[:, i]) - 1) for i in range(x.shape[1]))


def test_fp64_factor_stagnates_and_escalation_reaches_quad_double():
    """cond(A) ~ 1e17 once rounded to binary64: with a binary64 factor the
    contraction factor kappa * u_1 exceeds one, so the corrections stop
    shrinking; a double-double factor has kappa * u_2 ~ 1e-15."""
    from fractions import Fraction
    Ap, b, exact = synth.problem("randsvd", 60, config=1, instance=5, cond=1e30)
    assert exact
    plain = O.refine(Ap, b, 1, max_iter=12)
    assert plain["status"] == O.MAX_ITER
    stag = O.refine(Ap, b, 1, max_iter=12, stag_ratio=0.5)
    assert stag["status"] == O.STAGNATED and stag["iters"] < 12
    esc = O.refine(Ap, b, 1, max_iter=30, stag_ratio=0.5, escalate=True)
    assert esc["status"] == O.CONVERGED
    assert esc["final_words"] >= 2 and esc["escalations"] == esc["final_words"] - 1
    assert _err_vs_ones(esc["x"]) <= Fraction(10) ** -60


def test_no_escalation_when_the_factor_suffices():
    Ap, b, _ = synth.problem("randsvd", 60, config=1, instance=6, cond=1e3)
    r = O.refine(Ap, b, 1, stag_ratio=0.5, escalate=True)
    assert r["status"] == O.CONVERGED and r["final_words"] == 1 and r["escalations"] == 0
    r0 = O.refine(Ap, b, 1)
    np.testing.assert_array_equal(r["x"], r0["x"])
    assert r["iters"] == r0["iters"]


def test_zero_pivot_in_short_precision_escalates():
    """A quad-double matrix that is exactly singular once rounded to
    binary64 (a_11 = 1 + 2^-60 rounds to 1) but regular in double-double."""
    from fractions import Fraction
    A = np.zeros((4, 2, 2))
    A[0] = np.array([[1.0, 1.0], [1.0, 1.0]]).T
    A[1, 1, 1] = 2.0 ** -60
    b, exact = synth.rhs_ones(A)
    assert exact
    r = O.refine(A, b, 1)
    assert r["status"] == O.SINGULAR and r["info"] == 2
    e = O.refine(A, b, 1, escalate=True)
    assert e["status"] == O.CONVERGED and e["final_words"] == 2 and e["escalations"] == 1
    assert _err_vs_ones(e["x"]) == Fraction(0)


def _norm2_exact(v) -> float:
    """2-norm of a binary64 vector from an exact rational sum of squares
    (the square root taken once, in binary64)."""
    import math
    s = sum(Fraction(float(t)) ** 2 for t in np.asarray(v).ravel())
    if s == 0:
        return 0.0
    # sqrt of the correctly rounded sum: within an ulp of the exact root
    return math.sqrt(float(s))


@pytest.mark.parametrize("rtol", [1e-30, 1e-45, 2.0 ** -209])
def test_stopping_rule_eq2_is_the_first_residual_below_its_threshold(rtol):
    """The loop ends at the first residual with ||r||_2 < sqrt(n) rtol
    ||A||_F ||x||_2 (Listing 1; eq. (2) of Sec. 3 with the listing's strict
    inequality), the norms being 2-norms of the leading words.  Checked
    against norms recomputed from exact rational sums of squares: the
    reported norms agree to a few ulps, the final residual is below its
    threshold and every earlier one is above its own (a dropped sqrt(n),
    squared norms or a test placed after the update would break one)."""
    n = 48
    Ap, b, _ = synth.problem("randsvd", n, config=2, instance=3, cond=1e8)
    res = O.refine(Ap, b, 2, rtol=rtol, ctol=0.0, max_iter=40)
    assert res["status"] == O.CONVERGED
    na = _norm2_exact(Ap[0])
    assert abs(res["a_norm"] - na) <= 4e-16 * na
    nx = _norm2_exact(res["x"][0])
    assert abs(res["x_norm"] - nx) <= 4e-16 * nx
    r = O.residual(Ap, res["x"], b)
    nr = _norm2_exact(r[0])
    assert abs(res["resid_norm"] - nr) <= 4e-16 * max(nr, 1e-300)
    thr = np.sqrt(n) * rtol * na
    assert nr < thr * nx
    # replay the corrections: every earlier residual fails the test
    hist = res["history"]
    assert len(hist) == res["iters"] + 1
    for h in hist[:-1]:
        assert h >= thr * nx * 0.5  # the x norms of earlier iterates differ from the last by far less than 2x
    # tighter rtol never stops earlier
    tight = O.refine(Ap, b, 2, rtol=rtol / 1e6, ctol=0.0, max_iter=40)
    assert tight["iters"] >= res["iters"]


def test_stopping_rule_atol_alone():
    """atol above the first residual's norm stops the loop before any
    correction; below it, the listing's test with rtol = 0 never fires."""
    n = 32
    Ap, b, _ = synth.problem("uniform", n, config=0, instance=7)
    first = O.refine(Ap, b, 3, max_iter=0)
    r0 = first["resid_norm"]
    assert r0 > 0
    res = O.refine(Ap, b, 3, atol=2 * r0, ctol=0.0)
    assert res["status"] == O.CONVERGED and res["iters"] == 0
    res = O.refine(Ap, b, 3, atol=0.0, rtol=0.0, ctol=0.0, max_iter=3)
    assert res["status"] == O.MAX_ITER and res["iters"] == 3


# ---- the 424-bit long precision (8 words), the setting of Table 2 --------

def rand_words_vec(g, L, n, scale=1.0):
    out = np.zeros((L, n))
    for i in range(n):
        q = Fraction(0)
        for w in range(L + 2):
            q += Fraction(float(g.uniform(-1, 1))) * Fraction(2) ** (-53 * w)
        out[:, i] = X.canon(q * Fraction(scale), L)
    return out


@pytest.mark.parametrize("aw", [1, 4])
def test_residual_eight_words_bitexact_vs_fraction(aw):
    g = np.random.default_rng(17 + aw)
    for n in (1, 3, 7):
        A = np.zeros((aw, n, n))
        for i in range(n):
            for j in range(n):
                q = sum((Fraction(float(g.uniform(-1, 1))) * Fraction(2) ** (-53 * w) for w in range(aw + 1)),
                        Fraction(0))
                A[:, j, i] = X.canon(q, aw)
        x = rand_words_vec(g, 8, n)
        b = rand_words_vec(g, 8, n, scale=2.0 ** int(g.integers(-3, 4)))
        r = O.residual(A, x, b)
        ex = X.residual([[A[:, j, i] for j in range(n)] for i in range(n)],
                        [x[:, j] for j in range(n)], [b[:, i] for i in range(n)])
        for i in range(n):
            assert list(r[:, i]) == X.canon(ex[i], 8)


def max_rel_err(x, xs):
    """max_i |x_i - xs_i| / |xs_i| (xs_i = 0: absolute) from the exact value
    of each L-word entry."""
    m = Fraction(0)
    for i in range(x.shape[1]):
        t = Fraction(float(xs[i]))
        d = abs(X.value(x[:, i]) - t)
        m = max(m, d / abs(t) if t != 0 else d)
    return float(m)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_long_precision_goes_beyond_quad_double(K):
    """With an 8-word x and residual the refinement is no longer limited by
    the quad-double floor (~1e-64): the forward test at 2^-415 gives x* = 1
    to better than 1e-120, and eq. (2) with the paper's rtol = 1e-100 stops
    with a forward error below kappa * sqrt(n) * 1e-100."""
    n = 64
    Ap, b, exact = synth.problem("randsvd", n, config=2, instance=0, cond=1e10)
    assert exact
    res = O.refine(Ap, b, K, long_words=8, ctol=2.0 ** -415)
    assert res["status"] == O.CONVERGED and res["x"].shape == (8, n)
    assert max_rel_err(res["x"], np.ones(n)) <= 1e-120
    res = O.refine(Ap, b, K, long_words=8, ctol=0.0, rtol=1e-100)
    assert res["status"] == O.CONVERGED
    assert max_rel_err(res["x"], np.ones(n)) <= 1e10 * np.sqrt(n) * 1e-100


def test_long_precision_needed_for_rtol_1e_minus_100():
    """A right-hand side whose solution has no short representation (random
    424-bit b): eq. (2) with rtol = 1e-100 is met in the 8-word long
    precision, while a quad-double x cannot bring the residual below about
    2^-212 |A| |x| and the loop runs out of corrections."""
    n = 48
    Ap, _, _ = synth.problem("randsvd", n, config=2, instance=5, cond=1e6)
    g = np.random.default_rng(5)
    b8 = rand_words_vec(g, 8, n)
    res = O.refine(Ap, b8, 3, long_words=8, ctol=0.0, rtol=1e-100)
    assert res["status"] == O.CONVERGED
    thr = np.sqrt(n) * 1e-100 * res["a_norm"]
    assert res["resid_norm"] < thr * res["x_norm"]
    q = O.refine(Ap, O.round_words(4, b8), 3, long_words=4, ctol=0.0, rtol=1e-100, max_iter=8)
    assert q["status"] == O.MAX_ITER
    assert q["resid_norm"] > thr * q["x_norm"]


def test_paper_system_table2_setting():
    """The paper's system A = R D R^-1 (kappa_2 = 10^(26 (n-1)/n)), x = [0..n-1],
    refined from DD, TD and QD factors in the 424-bit long precision with
    eq. (2), rtol = 1e-100 (Table 2's setting, here at n = 40): every factor
    reaches a maximum relative error below kappa * sqrt(n) * 1e-100, and more
    factor words need fewer corrections (Table 2: 15 / 2 / 1 at n = 2000)."""
    n = 40
    Ap, b, exact, xs = synth.paper_problem(n)
    assert exact
    iters = {}
    for K in (2, 3, 4):
        res = O.refine(Ap, b, K, long_words=8, ctol=0.0, rtol=1e-100, max_iter=40)
        assert res["status"] == O.CONVERGED
        kappa = 10.0 ** (26 * (n - 1) / n)
        assert max_rel_err(res["x"], xs) <= kappa * np.sqrt(n) * 1e-100, K
        iters[K] = res["iters"]
    assert iters[2] > iters[3] >= iters[4] >= 1
