"""The bounded waits' timeout paths, forced from the host: the library's
test hook raises each wait's abort flag right after the reset, so every
poll gives up at once while every kernel still runs to its end on
in-bounds memory.  The stand-alone factorisation and substitution must
report info = -1, bnc_refine must return BNC_ERR_TIMEOUT (not a singular
status or an escalation), and with the hook off everything is bit-exact
again.
"""
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


@pytest.fixture
def hook(P):
    yield P.test_force_timeout
    P.test_force_timeout(0)


N, K = 200, 2


@pytest.fixture(scope="module")
def system():
    Ap, b, _ = synth.problem("uniform", N, config=0, instance=41)
    return Ap, b


def test_getrs_reports_timeout(P, hook, system):
    import torch
    Ap, b = system
    A = O.stage(K, Ap)
    LU, ipiv, _ = O.getrf(K, A)
    dA = dev(A)
    dipiv, dinfo = P.getrf(K, dA)
    assert int(host(dinfo)[0]) == 0
    bf = O.round_words(K, b)
    info = torch.full((1,), 7, dtype=torch.int64, device="cuda")
    say("getrs forced timeout")
    hook(2)
    P.getrs(K, dA, dipiv, dev(bf), info=info)
    assert int(host(info)[0]) == -1
    hook(0)
    dx = dev(bf)
    say("getrs after the hook")
    P.getrs(K, dA, dipiv, dx, info=info)
    assert int(host(info)[0]) == 0
    np.testing.assert_array_equal(host(dx), O.getrs(K, LU, ipiv, bf))


@pytest.mark.parametrize("oz", [0, 5])
def test_getrf_reports_timeout(P, hook, system, oz):
    Ap, _ = system
    A = O.stage(K, Ap)
    say("getrf forced timeout oz", oz)
    hook(1)
    dA = dev(A)
    _, dinfo = P.getrf_ozaki(K, oz, dA) if oz else P.getrf(K, dA)
    assert int(host(dinfo)[0]) == -1
    hook(0)
    dA = dev(A)
    say("getrf after the hook oz", oz)
    dipiv, dinfo = P.getrf_ozaki(K, oz, dA) if oz else P.getrf(K, dA)
    LU, ipiv, info = O.getrf_ozaki(K, A, oz) if oz else O.getrf(K, A)
    assert int(host(dinfo)[0]) == info == 0
    np.testing.assert_array_equal(host(dipiv), ipiv)
    np.testing.assert_array_equal(host(dA), LU)


@pytest.mark.parametrize("bits", [1, 2])
def test_refine_returns_timeout(P, hook, system, bits):
    Ap, b = system
    say("refine forced timeout bits", bits)
    hook(bits)
    with pytest.raises(P.BncError) as e:
        P.refine(dev(Ap), dev(b), K, escalate=True, stagnation_ratio=0.5)
    assert e.value.code == P.BNC_ERR_TIMEOUT
    hook(0)
    say("refine after the hook")
    out = P.refine(dev(Ap), dev(b), K)
    ref = O.refine(Ap, b, K)
    assert out["status"] == ref["status"] and out["iters"] == ref["iters"]
    np.testing.assert_array_equal(host(out["x"]), ref["x"])
