"""GPU parity of the 424-bit long precision (8 binary64 words for x, b and
the residual; the long precision of the paper's Table 2, Kouya 2021 Sec. 3):
the exact residual rounded to 8 words, and the refinement from DD/TD/QD
factors with the forward test near 2^-424 or with eq. (2) at the paper's
rtol = 1e-100, bit for bit against the oracle (x, corrections, status)."""
import math
import sys
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import synth
from helpers import dev, host
from oracle import exact as X

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_12550_amd as P
    return P


def rand_long(g, n, L=8, scale=1.0, spread=0):
    out = np.zeros((L, n))
    for i in range(n):
        e = int(g.integers(-spread, spread + 1)) if spread else 0
        q = Fraction(0)
        for w in range(L + 2):
            q += Fraction(float(g.uniform(-1, 1))) * Fraction(2) ** (-53 * w + e)
        out[:, i] = X.canon(q * Fraction(scale), L)
    return out


@pytest.mark.parametrize("aw", [1, 4])
@pytest.mark.parametrize("n", [1, 3, 65, 300])
def test_residual_eight_words_bitexact(P, aw, n):
    g = np.random.default_rng(70 + n + aw)
    if aw == 1:
        Ap = synth.planes(g.uniform(-1, 1, (n, n)))
    else:
        Ap, _, _ = synth.problem("randsvd_words", n, config=0, instance=n, cond=1e20) if n > 1 else \
            (np.array([[[0.75]], [[2.0 ** -60]], [[2.0 ** -120]], [[2.0 ** -180]]]), None, None)
    x = rand_long(g, n, spread=3)
    b = rand_long(g, n, scale=2.0 ** int(g.integers(-3, 4)))
    say("residual 8 words aw", aw, "n", n)
    r = O.residual(Ap, x, b)
    dr, flag = P.residual(dev(Ap), dev(x), dev(b))
    assert int(host(flag)[0]) == 0
    np.testing.assert_array_equal(host(dr), r)
    # near the solution: b - A x is tiny and cancels over many bins
    x1 = O.round_words(8, np.vstack([np.ones((1, n)), np.zeros((7, n))]))
    # A x1 rounded to quad-double: the residual is about 2^-212 of A x1
    b1 = O.extend(O.round_words(4, O.residual(Ap, -x1, np.zeros((8, n)))), 8)
    say("residual near the solution aw", aw, "n", n)
    dr, flag = P.residual(dev(Ap), dev(x1), dev(b1))
    np.testing.assert_array_equal(host(dr), O.residual(Ap, x1, b1))


CASES = [(1, "uniform", 64, 1.0), (2, "randsvd", 200, 1e10), (3, "randsvd", 300, 1e10), (4, "uniform", 130, 1.0)]


@pytest.mark.parametrize("K,kind,n,cond", CASES)
def test_refine_eight_words_forward_test_bitexact(P, K, kind, n, cond):
    Ap, b, exact = synth.problem(kind, n, config=2, instance=80 + K, cond=cond)
    assert exact
    b8 = O.extend(b, 8)
    kw = dict(long_words=8, ctol=2.0 ** -415)
    say("refine 8 words K", K, kind, n)
    ref = O.refine(Ap, b8, K, **kw)
    out = P.refine(dev(Ap), dev(b8), K, **kw)
    assert out["status"] == ref["status"] == O.CONVERGED
    assert out["iters"] == ref["iters"]
    np.testing.assert_array_equal(host(out["x"]), ref["x"])
    assert max(abs(math.fsum([ref["x"][0, i] - 1.0] + list(ref["x"][1:, i]))) for i in range(n)) <= 1e-120


@pytest.mark.parametrize("K,oz", [(2, 0), (3, 0), (4, 0), (2, 5), (3, 7)])
def test_paper_system_rtol_1e_minus_100_bitexact(P, K, oz):
    """Table 2's setting on the paper's system (here n = 300): eq. (2) with
    rtol = 1e-100, 8-word long precision, quad-double-word entries."""
    n = 300
    Ap, b, exact, xs = synth.paper_problem(n)
    assert exact
    b8 = O.extend(b, 8)
    kw = dict(long_words=8, ctol=0.0, rtol=1e-100, max_iter=40, ozaki=oz)
    say("paper system 8 words K", K, "ozaki", oz)
    ref = O.refine(Ap, b8, K, **kw)
    out = P.refine(dev(Ap), dev(b8), K, **kw)
    assert out["status"] == ref["status"] == O.CONVERGED
    assert out["iters"] == ref["iters"]
    np.testing.assert_array_equal(host(out["x"]), ref["x"])
    for f in ("resid_norm", "x_norm", "a_norm"):
        assert abs(out[f] - ref[f]) <= 1e-13 * abs(ref[f]), f
    assert out["resid_norm"] < math.sqrt(n) * 1e-100 * out["a_norm"] * out["x_norm"]


def test_general_rhs_needs_the_long_precision(P):
    """A 424-bit right-hand side: eq. (2) with rtol = 1e-100 is met with 8
    words and not with 4 (the loop runs out of corrections), on the GPU as
    in the oracle."""
    n = 96
    Ap, _, _ = synth.problem("randsvd", n, config=2, instance=90, cond=1e6)
    g = np.random.default_rng(90)
    b8 = rand_long(g, n)
    say("general rhs 8 words")
    ref = O.refine(Ap, b8, 3, long_words=8, ctol=0.0, rtol=1e-100)
    out = P.refine(dev(Ap), dev(b8), 3, long_words=8, ctol=0.0, rtol=1e-100)
    assert out["status"] == ref["status"] == O.CONVERGED and out["iters"] == ref["iters"]
    np.testing.assert_array_equal(host(out["x"]), ref["x"])
    b4 = O.round_words(4, b8)
    ref4 = O.refine(Ap, b4, 3, long_words=4, ctol=0.0, rtol=1e-100, max_iter=8)
    out4 = P.refine(dev(Ap), dev(b4), 3, long_words=4, ctol=0.0, rtol=1e-100, max_iter=8)
    assert out4["status"] == ref4["status"] == O.MAX_ITER
    np.testing.assert_array_equal(host(out4["x"]), ref4["x"])
