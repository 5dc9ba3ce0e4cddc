"""GPU parity of the refinement loop's stopping tests (Kouya 2021, Sec. 2,
Listing 1; eq. (2) of Sec. 3): the residual test ||r||_2 < sqrt(n) rtol
||A||_F ||x||_2 + atol alone (ctol = 0), together with the forward test,
and the absolute tolerance.  Status, corrections and every word of x must
equal the oracle's; the device norms that feed the test (||r||_2, ||x||_2,
||A||_F over leading words, summed in a fixed order) must agree with the
oracle's correctly rounded ones to a few ulps.
"""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from helpers import dev, host

pytestmark = pytest.mark.gpu

RTOL_QD = 2.0 ** -209  # eq. (2) at the quad-double unit roundoff


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_12550_amd as P
    return P


def check(P, Ap, b, K, **kw):
    ref = O.refine(Ap, b, K, **kw)
    out = P.refine(dev(Ap), dev(b), K, **kw)
    assert out["status"] == ref["status"], (out["status"], ref["status"])
    assert out["iters"] == ref["iters"], (out["iters"], ref["iters"])
    np.testing.assert_array_equal(host(out["x"]), ref["x"])
    for f in ("resid_norm", "x_norm", "a_norm"):
        assert abs(out[f] - ref[f]) <= 1e-13 * max(abs(ref[f]), 1e-300), (f, out[f], ref[f])
    return out, ref


CASES = [("uniform", 200, 0, 1.0), ("randsvd", 300, 1, 1e10), ("randsvd", 130, 1, 1e15)]


@pytest.mark.parametrize("kind,n,config,cond", CASES)
@pytest.mark.parametrize("K", [2, 3])
def test_residual_test_alone(P, kind, n, config, cond, K):
    say("eq2 alone", kind, n, cond, "K", K)
    Ap, b, _ = synth.problem(kind, n, config=config, instance=31, cond=cond)
    out, ref = check(P, Ap, b, K, rtol=RTOL_QD, ctol=0.0)
    assert ref["status"] == O.CONVERGED
    # the loop ended on eq. (2): the last residual is below its threshold
    assert out["resid_norm"] < np.sqrt(n) * RTOL_QD * out["a_norm"] * out["x_norm"]


@pytest.mark.parametrize("K", [2, 3, 4])
def test_residual_and_forward_tests_together(P, K):
    n = 257
    say("eq2 + forward test K", K)
    Ap, b, _ = synth.problem("randsvd", n, config=1, instance=32, cond=1e12)
    check(P, Ap, b, K, rtol=RTOL_QD, ctol=2.0 ** -208)


def test_residual_test_stops_the_loop_first(P):
    """A loose rtol: eq. (2) fires corrections before the forward test
    would, with both on."""
    n = 200
    Ap, b, _ = synth.problem("randsvd", n, config=1, instance=33, cond=1e10)
    say("eq2 first")
    fwd = O.refine(Ap, b, 2, rtol=0.0, ctol=2.0 ** -208)
    out, ref = check(P, Ap, b, 2, rtol=1e-40, ctol=2.0 ** -208)
    assert ref["status"] == O.CONVERGED and ref["iters"] < fwd["iters"]
    assert out["resid_norm"] < np.sqrt(n) * 1e-40 * out["a_norm"] * out["x_norm"]


def test_absolute_tolerance(P):
    n = 96
    Ap, b, _ = synth.problem("uniform", n, config=0, instance=34)
    first = O.refine(Ap, b, 3, max_iter=0)
    say("atol")
    out, ref = check(P, Ap, b, 3, atol=2 * first["resid_norm"], ctol=0.0)
    assert ref["iters"] == 0 and ref["status"] == O.CONVERGED
    check(P, Ap, b, 3, atol=0.0, rtol=0.0, ctol=0.0, max_iter=3)


def test_split_form_with_residual_test(P):
    n = 300
    Ap, b, _ = synth.problem("randsvd", n, config=2, instance=35, cond=1e10)
    say("eq2 split form")
    out, ref = check(P, Ap, b, 2, rtol=RTOL_QD, ctol=0.0, ozaki=5)
    assert ref["status"] == O.CONVERGED
