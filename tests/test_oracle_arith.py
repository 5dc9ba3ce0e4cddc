"""Pins for the oracle's error-free transformations and K-word primitives.

Everything here is checked against exact rational arithmetic (Fraction) or
against plain binary64 (K = 1), never against the oracle itself.  The bounds
are in units of 2^(-53 K), the precision the paper assigns to DD/TD/QD
(106/159/212 bits, Table 1 of Kouya 2021).  For the double-double product
the level-1 sum of three partial products rounds twice and a_1 b_1 is
dropped, about 8 units in all; the same constant is used for every K.  A dropped partial product, a
wrong sign or a lost rounding error costs a factor ~2^53 and fails them.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from oracle.exact import canon, value

U = {K: 2.0 ** (-53 * K) for K in (1, 2, 3, 4)}


def rand_words(g, K, n, spread=3, cancel_with=None):
    """Random canonical K-word numbers: greedy rounding of random rationals
    carrying a few words more than K, exponents in [-spread, spread]."""
    out = np.zeros((K, n))
    for i in range(n):
        e = int(g.integers(-spread, spread + 1))
        q = Fraction(0)
        for w in range(K + 2):
            q += Fraction(float(g.uniform(-1, 1))) * Fraction(2) ** (-53 * w + e)
        out[:, i] = canon(q, K)
    return out


def adversarial_doubles(g, n):
    e = g.integers(-60, 60, size=n)
    m = g.uniform(-1, 1, size=n)
    x = np.ldexp(m, e)
    x[::7] = 0.0
    x[1::11] = -x[1::11]
    x[2::13] = np.ldexp(1.0, e[2::13])          # powers of two
    x[3::17] = np.nextafter(1.0, 2.0)           # 1 + ulp
    return x


def test_two_sum_exact():
    g = np.random.default_rng(11)
    a = adversarial_doubles(g, 4000)
    b = np.concatenate([adversarial_doubles(g, 3000), -a[:1000]])
    s, e = O.two_sum(a, b)
    for i in range(a.size):
        assert Fraction(s[i]) + Fraction(e[i]) == Fraction(a[i]) + Fraction(b[i])
        assert s[i] == float(Fraction(a[i]) + Fraction(b[i]))  # s = RN(a+b)


def test_two_prod_exact():
    g = np.random.default_rng(12)
    a = adversarial_doubles(g, 4000)
    b = adversarial_doubles(g, 4000)[::-1].copy()
    p, e = O.two_prod(a, b)
    for i in range(a.size):
        assert Fraction(p[i]) + Fraction(e[i]) == Fraction(a[i]) * Fraction(b[i])
        assert p[i] == float(Fraction(a[i]) * Fraction(b[i]))


def test_k1_is_plain_binary64():
    """With one word every primitive is the plain IEEE operation."""
    g = np.random.default_rng(13)
    a, b, c = (adversarial_doubles(g, 3000)[None, :] for _ in range(3))
    a[a == 0] = 0.5
    np.testing.assert_array_equal(O.add(1, a, b), a + b)
    np.testing.assert_array_equal(O.mul(1, a, b), a * b)
    np.testing.assert_array_equal(O.fms(1, c, a, b), c - a * b)
    np.testing.assert_array_equal(O.recip(1, a), 1.0 / a)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_primitive_error_bounds(K):
    g = np.random.default_rng(100 + K)
    n = 1500
    a, b, c = rand_words(g, K, n), rand_words(g, K, n), rand_words(g, K, n)
    # a third of the cases cancel c against a*b down to 2^-40 relative
    ab = O.mul(K, a, b)
    c[:, : n // 3] = ab[:, : n // 3]
    c[0, : n // 3] *= 1 + 2.0 ** -40
    f, m, s, r = O.fms(K, c, a, b), O.mul(K, a, b), O.add(K, a, b), O.recip(K, a)
    u = Fraction(U[K])
    for i in range(n):
        av, bv, cv = value(a[:, i]), value(b[:, i]), value(c[:, i])
        assert abs(value(f[:, i]) - (cv - av * bv)) <= 8 * u * (abs(cv) + abs(av * bv))
        assert abs(value(m[:, i]) - av * bv) <= 8 * u * abs(av * bv)
        assert abs(value(s[:, i]) - (av + bv)) <= 4 * u * (abs(av) + abs(bv))
        assert abs(value(r[:, i]) * av - 1) <= 16 * u


@pytest.mark.parametrize("K", [2, 3, 4])
def test_outputs_nonoverlapping(K):
    g = np.random.default_rng(200 + K)
    n = 2000
    a, b, c = rand_words(g, K, n), rand_words(g, K, n), rand_words(g, K, n)
    for out in (O.fms(K, c, a, b), O.mul(K, a, b), O.add(K, a, b), O.recip(K, a)):
        for w in range(K - 1):
            hi, lo = np.abs(out[w]), np.abs(out[w + 1])
            assert np.all(lo <= np.ldexp(hi, -51)), (K, w)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_identities(K):
    """x*1 = x, x+0 = x, c - x*0 = c, exactly, on canonical inputs."""
    g = np.random.default_rng(300 + K)
    n = 1000
    a, c = rand_words(g, K, n), rand_words(g, K, n)
    one = np.zeros((K, n))
    one[0] = 1.0
    zero = np.zeros((K, n))
    np.testing.assert_array_equal(O.mul(K, a, one), a)
    np.testing.assert_array_equal(O.add(K, a, zero), a)
    np.testing.assert_array_equal(O.fms(K, c, a, zero), c)
    neg = -a
    np.testing.assert_array_equal(O.add(K, a, neg), zero)


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_exact_rounding_matches_fraction(K):
    """The exact accumulator used by the residual rounds like Fraction."""
    g = np.random.default_rng(400 + K)
    for trial in range(60):
        m = int(g.integers(1, 40))
        p = adversarial_doubles(g, m)
        q = adversarial_doubles(g, m)
        s = g.choice([-1, 1], size=m).astype(np.int32)
        got, bad = O.exact_round(K, p, q, s)
        exact = sum((int(s[t]) * Fraction(p[t]) * Fraction(q[t]) for t in range(m)), Fraction(0))
        assert not bad
        assert list(got) == canon(exact, K)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_key_order_is_magnitude_order_on_canonical(K):
    g = np.random.default_rng(500 + K)
    n = 2000
    a = rand_words(g, K, n, spread=1)
    b = a.copy()
    # perturb in a random word so that many pairs share leading words
    w = g.integers(0, K, size=n)
    for i in range(n):
        b[:, i] = canon(value(a[:, i]) * (1 + Fraction(float(g.uniform(-1, 1))) * Fraction(2) ** (-53 * int(w[i]) - 3)), K)
    b[:, ::5] = -b[:, ::5]
    gt = O.key_gt(K, a, b)
    for i in range(n):
        assert gt[i] == (abs(value(a[:, i])) > abs(value(b[:, i])))


def _spread_words(g, m, n, gap):
    """m-word values whose words are random binary64 numbers `gap` bits
    apart (gap < 53: overlapping words, not canonical)."""
    out = np.zeros((m, n))
    for i in range(n):
        e = int(g.integers(-20, 21))
        for w in range(m):
            out[w, i] = np.ldexp(g.uniform(-1, 1), e - gap * w)
    return out


@pytest.mark.parametrize("m", [2, 3, 4])
def test_round_words_canonical_input_is_greedy_rounding(m):
    """Long -> short conversion of Listing 1 (the K-word copies of A, b and
    every residual): m canonical words rounded to K < m words equal the
    canonical K-word rounding of their exact value (w0 = RN(v), w1 = RN(v -
    w0), ...), bit for bit.  Dropping, mis-signing or double-rounding any
    folded word breaks this."""
    g = np.random.default_rng(600 + m)
    src = rand_words(g, m, 1500, spread=30)
    for K in range(1, m):
        out = O.round_words(K, src)
        for i in range(src.shape[1]):
            assert list(out[:, i]) == canon(value(src[:, i]), K), (m, K, i)


@pytest.mark.parametrize("m", [3, 4])
@pytest.mark.parametrize("gap", [30, 45, 53, 60])
def test_round_words_general_input_bound(m, gap):
    """Non-canonical m-word inputs (overlapping words, or the last two words
    nearly cancelling): the K-word result is within 2^(-53K) |v| of the
    exact value v for every K < m, and K = m keeps the value exactly."""
    g = np.random.default_rng(700 + 10 * m + gap)
    src = _spread_words(g, m, 1200, gap)
    src[m - 1, ::3] = -src[m - 2, ::3] * (1 - 2.0 ** -30)   # trailing words cancel
    u = {K: Fraction(2) ** (-53 * K) for K in range(1, 5)}
    for K in range(1, m + 1):
        out = O.round_words(K, src)
        for i in range(src.shape[1]):
            v = value(src[:, i])
            if K == m:
                assert value(out[:, i]) == v
            else:
                assert abs(value(out[:, i]) - v) <= u[K] * abs(v), (m, K, gap, i)


def test_round_words_widening_is_exact():
    """Short -> long (K >= m): the value is kept and the extra words are 0."""
    g = np.random.default_rng(800)
    src = rand_words(g, 2, 500)
    out = O.round_words(4, src)
    np.testing.assert_array_equal(out[2:], 0.0)
    for i in range(src.shape[1]):
        assert value(out[:, i]) == value(src[:, i])


def _exact_sqrt_sum_sq(v):
    """sqrt(sum v_i^2) of binary64 values to about 120 bits, from the exact
    rational sum of squares (integer square root of the scaled sum)."""
    import math
    s = sum((Fraction(float(x)) ** 2 for x in v), Fraction(0))
    if s == 0:
        return Fraction(0)
    # s = p / q; sqrt(s) ~ isqrt(p * q * 4^t) / (q * 2^t)
    t = 130
    return Fraction(math.isqrt(s.numerator * s.denominator * 4 ** t), s.denominator * 2 ** t)


def test_norm2_against_exact():
    """The 2-norm of Listing 1's stopping test (||r||_2, ||x||_2, ||A||_F of
    leading words): the squares of the scaled entries are rounded once each,
    summed with correct rounding and square-rooted once, so the result is
    within 2 ulp (2^-51 relative) of the exact norm, also for entries near
    the overflow and underflow thresholds."""
    g = np.random.default_rng(900)
    cases = [np.array([3.0, 4.0]), np.array([0.0, -0.0]), np.array([-7.5]), np.array([1e300, 1e300]),
             np.array([1e-300, 3e-310, -2e-300]), np.array([2.0 ** 600, -(2.0 ** 601)])]
    for n in (1, 2, 17, 256, 4096):
        cases.append(g.uniform(-1, 1, size=n) * 2.0 ** int(g.integers(-900, 900)))
        cases.append(adversarial_doubles(g, n))
    for v in cases:
        got = O.norm2(v)
        ref = _exact_sqrt_sum_sq(v)
        if ref == 0:
            assert got == 0.0
            continue
        assert abs(Fraction(got) - ref) <= Fraction(2) ** -51 * ref, (v[:4], got, float(ref))
    assert O.norm2(np.array([3.0, 4.0])) == 5.0
    assert O.norm2(np.array([-7.5])) == 7.5


# ---- the 424-bit long precision (8 words; Table 2 of Kouya 2021) -----------

def test_eight_word_add_bound_and_identities():
    """x <- x + z of the refinement in the 8-word long precision: within
    4 * 2^-424 (|a| + |b|) of the exact sum (Fraction), non-overlapping
    words, and exact identities; half the cases add a correction 2^-60 to
    2^-300 the size of x, as the refinement does."""
    g = np.random.default_rng(950)
    K, n = 8, 600
    a = rand_words(g, K, n)
    b = rand_words(g, K, n)
    b[:, ::2] = np.ldexp(b[:, ::2], -g.integers(60, 300, size=b[:, ::2].shape[1]))
    s = O.add(K, a, b)
    u = Fraction(2) ** (-53 * K)
    for i in range(n):
        av, bv = value(a[:, i]), value(b[:, i])
        assert abs(value(s[:, i]) - (av + bv)) <= 4 * u * (abs(av) + abs(bv)), i
    for w in range(K - 1):
        assert np.all(np.abs(s[w + 1]) <= np.ldexp(np.abs(s[w]), -51))
    np.testing.assert_array_equal(O.add(K, a, np.zeros((K, n))), a)
    np.testing.assert_array_equal(O.add(K, a, -a), np.zeros((K, n)))


def test_eight_word_to_short_rounding_is_greedy():
    """The 424-bit residual rounded to the factor's K words (the listing's
    long -> short conversion) is the canonical K-word rounding of its exact
    value, for every K < 8, and K = 8 keeps it exactly."""
    g = np.random.default_rng(951)
    src = rand_words(g, 8, 400, spread=40)
    for K in (1, 2, 3, 4, 8):
        out = O.round_words(K, src)
        for i in range(src.shape[1]):
            if K == 8:
                assert value(out[:, i]) == value(src[:, i])
            else:
                assert list(out[:, i]) == canon(value(src[:, i]), K), (K, i)


def test_exact_rounding_to_eight_words_matches_fraction():
    g = np.random.default_rng(952)
    for trial in range(40):
        m = int(g.integers(1, 40))
        p = adversarial_doubles(g, m)
        q = adversarial_doubles(g, m)
        s = g.choice([-1, 1], size=m).astype(np.int32)
        got, bad = O.exact_round(8, p, q, s)
        exact = sum((int(s[t]) * Fraction(p[t]) * Fraction(q[t]) for t in range(m)), Fraction(0))
        assert not bad
        assert list(got) == canon(exact, 8)
