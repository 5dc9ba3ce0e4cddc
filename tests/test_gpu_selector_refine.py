"""The learned precision choice as a library path: bnc_refine with
factor_words = BNC_AUTO computes the system's 24 features and runs the
network itself, factors with the predicted number of words and escalates
on stagnation.  The choice must equal the argmax of the stand-alone entry
points (bnc_features + bnc_mlp_forward) on the same system, and the refined
solution, corrections and status must equal bnc_refine started at that
precision, bit for bit (and the oracle's, for a sample)."""
import os
import sys

import numpy as np
import pytest

import oracle as O
import synth
from helpers import dev, host

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_12550_amd as P
    return P


@pytest.fixture(scope="module")
def net(P):
    from paper_2107_12550_amd import selector as SEL
    return SEL.load(os.path.join(ROOT, "paper_2107_12550_amd", "selector_model.npz"))


def test_auto_matches_the_separate_entry_points(P, net):
    import torch
    As, bs, exact, conds = synth.batch(48, 32, 512, 1.0, 60.0, config=8, words_above=1e15)
    dA = [torch.from_numpy(a).cuda() for a in As]
    db = [torch.from_numpy(b).cuda() for b in bs]
    F = P.features(dA, db)
    cls = torch.argmax(net.forward(F)[:, :4], dim=1).cpu().numpy()
    say("predicted classes", np.bincount(cls, minlength=4).tolist())
    assert len(set(cls.tolist())) >= 2
    kw = dict(escalate=True, stagnation_ratio=0.5, ctol=2.0 ** -150)
    for i in range(len(As)):
        out = P.refine(dA[i], db[i], P.BNC_AUTO, selector=net, **kw)
        assert out["first_words"] == cls[i] + 1, (i, out["first_words"], cls[i])
        ref = P.refine(dA[i], db[i], int(cls[i]) + 1, **kw)
        assert out["status"] == ref["status"] and out["iters"] == ref["iters"]
        assert out["final_words"] == ref["final_words"] and out["escalations"] == ref["escalations"]
        np.testing.assert_array_equal(host(out["x"]), host(ref["x"]))
        if i % 12 == 0 and As[i].shape[-1] <= 300:
            o = O.refine(As[i], bs[i], int(cls[i]) + 1, escalate=True, stag_ratio=0.5, ctol=2.0 ** -150)
            assert o["status"] == out["status"] and o["iters"] == out["iters"]
            np.testing.assert_array_equal(host(out["x"]), o["x"])


def test_auto_above_the_feature_limit_starts_at_two_words(P, net):
    n = 600
    Ap, b, _ = synth.problem("randsvd", n, config=8, instance=1, cond=1e8)
    out = P.refine(dev(Ap), dev(b), P.BNC_AUTO, selector=net, escalate=True, stagnation_ratio=0.5)
    assert out["first_words"] == 2 and out["status"] == P.BNC_CONVERGED
    ref = O.refine(Ap, b, 2, escalate=True, stag_ratio=0.5)
    np.testing.assert_array_equal(host(out["x"]), ref["x"])


def test_auto_needs_the_network(P):
    import torch
    Ap, b, _ = synth.problem("uniform", 16, config=8, instance=2)
    with pytest.raises(P.BncError):
        P.refine(torch.from_numpy(Ap).cuda(), torch.from_numpy(b).cuda(), P.BNC_AUTO)
