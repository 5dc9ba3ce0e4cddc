"""The direct-method sweep (no refinement) at n = 1024: double-double,
triple-double and quad-double getrf + getrs on randsvd systems with
binary64 entries (cond 1e3 and 1e15) and quad-double-word entries (cond
1e30), bit for bit against the oracle: pivots, info, every word of the
factor and of the solution.  The forward error against the exact solution
(all ones) must stay within the direct method's reach, a small multiple of
cond * u_K (Sec. 3, Table 1's pattern: more words, fewer lost digits)."""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from helpers import dev, host

pytestmark = pytest.mark.gpu

N = 1024
U = {2: 2.0 ** -104, 3: 2.0 ** -157, 4: 2.0 ** -209}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_12550_amd as P
    return P


@pytest.fixture(scope="module", autouse=True)
def all_threads():
    say("oracle threads", O.set_threads(0))


CASES = [(1e3, 2), (1e3, 3), (1e15, 3), (1e15, 4), (1e30, 4)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("cond,K", CASES)
def test_sweep_direct_method_bitexact(P, cond, K):
    kind = "randsvd" if cond <= 1e15 else "randsvd_words"
    Ap, b, exact = synth.problem(kind, N, config=1, instance=N, cond=cond)
    assert exact
    A0 = O.stage(K, Ap)
    say("oracle getrf/getrs n", N, "cond", cond, "K", K)
    LUo, ipo, info_o = O.getrf(K, A0)
    xo = O.getrs(K, LUo, ipo, O.round_words(K, b))
    say("gpu getrf/getrs n", N, "cond", cond, "K", K)
    dA = dev(A0)
    dipiv, dinfo = P.getrf(K, dA)
    assert int(host(dinfo)[0]) == info_o == 0
    np.testing.assert_array_equal(host(dipiv), ipo)
    np.testing.assert_array_equal(host(dA), LUo)
    dx = dev(O.round_words(K, b))
    P.getrs(K, dA, dipiv, dx)
    x = host(dx)
    np.testing.assert_array_equal(x, xo)
    err = float(np.max(np.abs(np.sum(np.vstack([x[0] - 1.0, x[1:]]), axis=0))))
    say("max |x - 1|", err, "cond * u_K", cond * U[K])
    assert err <= 1e4 * cond * U[K] + 1e-300
