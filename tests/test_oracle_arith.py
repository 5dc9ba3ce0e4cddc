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
