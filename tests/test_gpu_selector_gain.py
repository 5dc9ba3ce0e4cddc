"""What the trained precision selector gains over the method without it.

The shipped network (trained on systems the method labelled itself: n 32
to 512, cond 10^U(1, 60), quad-double-word entries above cond 1e15) picks
the factor precision of each system of a fresh held-out stream of the same
law (seed stream 7, never seen in training); the selector path is
features + network + batched refinement from the predicted precision,
escalating when the loop itself reports stagnation or no convergence.  The
method without it is escalate-on-stagnation from one word.  Both must bring
every system to convergence, and every converged solution must be within
1e-45 of the exact solution (checked afterwards; it decides nothing); the
selector must need fewer batched refinements (no wasted binary64 attempts)
and less refinement time.  Its end-to-end time, features and inference
included, is reported next to the escalation rule and a fixed
double-double start."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_selector_beats_escalation_on_held_out_systems():
    import os

    import torch

    from paper_2107_12550_amd import selector as SEL
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    net = SEL.load(os.path.join(root, "paper_2107_12550_amd", "selector_model.npz"))
    N = 1024
    As, bs, exact, _ = synth.batch(N, 32, 512, 1.0, 60.0, config=7, workers=min(16, os.cpu_count() or 1),
                                   words_above=1e15)
    assert all(exact)
    dA = [torch.from_numpy(a).cuda() for a in As]
    db = [torch.from_numpy(b).cuda() for b in bs]
    say("selector warm-up")
    SEL.evaluate(net, dA, db)
    say("selector vs escalation")
    r = SEL.evaluate(net, dA, db)
    say(r)
    assert r["baseline_solved"] == r["selector_solved"] == r["dd_solved"] == N
    assert r["baseline_wrong"] == r["selector_wrong"] == r["dd_wrong"] == 0
    assert r["selector_attempts"] < r["baseline_attempts"]
    assert r["fallback_fraction"] <= 0.05
    lab = SEL.label(dA, db)
    cls, _ = SEL.predict(net, SEL.bnc.features(dA, db))
    acc = float(np.mean(cls == lab["cls"]))
    majority = float(np.bincount(lab["cls"], minlength=4).max()) / len(dA)
    say("accuracy", acc, "majority class", majority)
    assert acc > majority + 0.05
    assert r["selector_solve_ms"] < 0.9 * r["baseline_ms"]
    say("end to end: selector", r["selector_ms"], "ms, escalation from one word", r["baseline_ms"],
        "ms, fixed double-double start", r["dd_ms"], "ms")
