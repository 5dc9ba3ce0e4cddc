"""GPU parity of the stagnation test and precision escalation (bnc_refine
with stagnation_ratio / escalate) against the oracle's refine: statuses,
the final factor precision, the number of escalations and corrections,
and the solution words must all be identical."""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from helpers import dev, host

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


def check(P, Ap, b, K, **kw):
    ozaki = kw.pop("ozaki", 0)
    ref = O.refine(Ap, b, K, ozaki=ozaki, escalate=kw.get("escalate", False),
                   stag_ratio=kw.get("stagnation_ratio", 0.0), max_iter=kw.get("max_iter", 30))
    out = P.refine(dev(Ap), dev(b), K, ozaki=ozaki, **kw)
    assert out["status"] == ref["status"]
    assert out["iters"] == ref["iters"]
    assert out["final_words"] == ref["final_words"] and out["escalations"] == ref["escalations"]
    if ref["status"] in (O.CONVERGED, O.MAX_ITER, O.STAGNATED):
        np.testing.assert_array_equal(host(out["x"]), ref["x"])
    return out


@pytest.mark.parametrize("n", [60, 150])
def test_stagnation_and_escalation_bitexact(P, n):
    Ap, b, _ = synth.problem("randsvd", n, config=1, instance=5, cond=1e30)
    say("stagnated n", n)
    out = check(P, Ap, b, 1, max_iter=12, stagnation_ratio=0.5)
    assert out["status"] == P.BNC_STAGNATED
    say("escalated n", n)
    out = check(P, Ap, b, 1, stagnation_ratio=0.5, escalate=True)
    assert out["status"] == P.BNC_CONVERGED and out["final_words"] >= 2
    say("escalated from split form n", n)
    check(P, Ap, b, 2, ozaki=2, stagnation_ratio=0.5, escalate=True)


def test_zero_pivot_in_short_precision_escalates(P):
    A = np.zeros((4, 2, 2))
    A[0] = np.array([[1.0, 1.0], [1.0, 1.0]]).T
    A[1, 1, 1] = 2.0 ** -60
    b, _ = synth.rhs_ones(A)
    say("singular in binary64")
    out = check(P, A, b, 1)
    assert out["status"] == P.BNC_SINGULAR
    out = check(P, A, b, 1, escalate=True)
    assert out["status"] == P.BNC_CONVERGED and out["final_words"] == 2


def test_no_escalation_when_not_needed(P):
    Ap, b, _ = synth.problem("randsvd", 130, config=1, instance=6, cond=1e3)
    say("well conditioned")
    out = check(P, Ap, b, 2, stagnation_ratio=0.5, escalate=True)
    assert out["escalations"] == 0 and out["final_words"] == 2
