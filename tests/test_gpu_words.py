"""Matrices stored in quad-double words (condition numbers that binary64
entries cannot carry, 1e25 and 1e30): the refined solution is bit-identical
to the oracle's and reaches the exact solution (all ones) to 1e-60, in the
K-word and the split forms."""
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


@pytest.mark.parametrize("K,oz,n,cond", [(3, 0, 130, 1e25), (3, 5, 200, 1e25), (4, 0, 96, 1e30), (2, 0, 70, 1e25)])
def test_refine_word_entries_bitexact(P, K, oz, n, cond):
    Ap, b, exact = synth.problem("randsvd_words", n, config=12, instance=n, cond=cond)
    assert exact and Ap.shape[0] == 4
    ref = O.refine(Ap, b, K, ozaki=oz, escalate=(K == 2), stag_ratio=0.5 if K == 2 else 0.0)
    say("refine words K", K, "oz", oz, "n", n, "cond", cond, "oracle status", ref["status"], "iters", ref["iters"])
    out = P.refine(dev(Ap), dev(b), K, ozaki=oz, escalate=(K == 2), stagnation_ratio=0.5 if K == 2 else 0.0)
    assert out["status"] == ref["status"] and out["iters"] == ref["iters"]
    np.testing.assert_array_equal(host(out["x"]), ref["x"])
    if ref["status"] == O.CONVERGED:
        x = ref["x"]
        assert float(np.max(np.abs((x[0] - 1.0) + x[1] + x[2] + x[3]))) <= 1e-60


@pytest.mark.parametrize("K,oz", [(2, 0), (3, 0), (3, 5)])
def test_paper_system_bitexact(P, K, oz):
    """The paper's test system (Sec. 3: A = R D R^-1, d_i = 10^(-26 (i-1)/n),
    x = [0..n-1]) at n = 100 (two panels and a ragged one): the refined
    solution, status and correction count equal the oracle's bit for bit, and
    the solution is x to quad-double accuracy."""
    Ap, b, exact, xs = synth.paper_problem(100, instance=3)
    assert exact
    say("paper system K", K, "oz", oz)
    ref = O.refine(Ap, b, K, ozaki=oz)
    out = P.refine(dev(Ap), dev(b), K, ozaki=oz)
    assert out["status"] == ref["status"] == O.CONVERGED and out["iters"] == ref["iters"]
    x = host(out["x"])
    np.testing.assert_array_equal(x, ref["x"])
    err = np.abs((x[0] - xs) + x[1:].sum(axis=0)) / np.maximum(xs, 1.0)
    assert err.max() < 1e-60
