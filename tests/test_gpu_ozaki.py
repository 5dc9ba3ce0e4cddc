"""GPU parity of the split (Ozaki) trailing update: bnc_getrf_ozaki and
bnc_refine with ozaki_slices against the oracle's getrf_ozaki / refine.

Every group sum of slice products is exact, so the matrix-core tiles give
exactly the numbers of the oracle's plain loops and the K-word combination
follows the same order: factors, pivots and refined solutions must be equal
bit for bit.
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


CASES = [(1, 3, 1), (2, 6, 5), (3, 8, 64), (4, 11, 65), (3, 8, 130), (2, 5, 200), (3, 12, 129), (4, 9, 257),
         (3, 1, 150), (2, 2, 300), (1, 4, 190)]


@pytest.mark.parametrize("K,s,n", CASES)
def test_getrf_ozaki_bitexact(P, K, s, n):
    kind = "uniform" if n % 2 else "randsvd"
    Ap, _, _ = synth.problem(kind, n, config=0, instance=300 + n, cond=1e12)
    A = O.stage(K, Ap)
    LU, ipiv, info = O.getrf_ozaki(K, A, s)
    say("getrf_ozaki K", K, "s", s, "n", n)
    dA = dev(A)
    dipiv, dinfo = P.getrf_ozaki(K, s, dA)
    np.testing.assert_array_equal(host(dipiv), ipiv)
    assert int(host(dinfo)[0]) == info
    np.testing.assert_array_equal(host(dA), LU)


def test_getrf_ozaki_singular_and_constructed(P):
    g = np.random.default_rng(31)
    n = 150
    L = np.tril(g.integers(-7, 8, (n, n)) / 8.0, -1) + np.eye(n)
    U = np.triu(g.integers(-9, 10, (n, n)).astype(float), 1)
    U += np.diag(g.choice([-4.0, -2.0, -1.0, 1.0, 2.0, 4.0], n))
    A = (L @ U)[np.argsort(g.permutation(n))]
    for K, s in ((2, 2), (3, 8)):
        Ap = np.zeros((K, n, n))
        Ap[0] = A.T
        LU, ipiv, _ = O.getrf_ozaki(K, Ap, s)
        say("constructed K", K, "s", s)
        dA = dev(Ap)
        dipiv, dinfo = P.getrf_ozaki(K, s, dA)
        np.testing.assert_array_equal(host(dA), LU)
        np.testing.assert_array_equal(host(dipiv), ipiv)
        assert int(host(dinfo)[0]) == 0
    # exactly singular: a zero on U's diagonal beyond the first panel keeps
    # every intermediate value an exact dyadic, so column 100 of the Schur
    # complement is exactly zero
    U[100, 100] = 0.0
    A = (L @ U)[np.argsort(g.permutation(n))]
    Ap = np.zeros((3, n, n))
    Ap[0] = A.T
    LU, ipiv, info = O.getrf_ozaki(3, Ap, 6)
    assert info == 101
    say("singular")
    dA = dev(Ap)
    dipiv, dinfo = P.getrf_ozaki(3, 6, dA)
    assert int(host(dinfo)[0]) == info
    np.testing.assert_array_equal(host(dipiv), ipiv)
    np.testing.assert_array_equal(host(dA), LU)


@pytest.mark.parametrize("K,s,n,cond", [(2, 5, 130, 1e8), (3, 8, 200, 1e12), (4, 11, 96, 1e20), (3, 3, 140, 1e4)])
def test_refine_ozaki_bitexact(P, K, s, n, cond):
    Ap, b, _ = synth.problem("randsvd", n, config=1, instance=60 + n, cond=cond)
    ref = O.refine(Ap, b, K, ozaki=s)
    say("refine ozaki K", K, "s", s, "n", n)
    out = P.refine(dev(Ap), dev(b), K, ozaki=s)
    assert out["status"] == ref["status"] and out["iters"] == ref["iters"]
    np.testing.assert_array_equal(host(out["x"]), ref["x"])


def test_ozaki_argument_errors(P):
    import torch
    A = torch.zeros((3, 4, 4), dtype=torch.float64, device="cuda")
    for K, s, code in ((3, 0, -2), (3, 13, -2), (5, 4, -1), (0, 4, -1)):
        with pytest.raises(P.BncError, match=f"code {code}"):
            P.getrf_ozaki(K, s, A)
    with pytest.raises(P.BncError):
        P.refine(torch.zeros((1, 4, 4), dtype=torch.float64, device="cuda"),
                 torch.zeros((4, 4), dtype=torch.float64, device="cuda"), 3, ozaki=13)


def test_split_range_reported_and_refinement_falls_back(P):
    """Below the split scheme's exact range (U12 column scales under
    oz_emin, the matrix scaled by 2^(oz_emin - 20)) the split factorisation
    reports info = -3, as the oracle's does; bnc_refine then factors in the
    plain form, bit for bit the oracle's refinement (which does the same),
    and bnc_refine_async ends with BNC_SPLIT_RANGE.  Scaled well above the
    bound nothing is reported and the factors equal the oracle's."""
    import torch
    K, s, n = 2, 4, 100
    Ap, b, exact = synth.problem("uniform", n, config=1, instance=77)
    assert exact
    e = O.oz_emin(K, s)
    low, ok = np.ldexp(Ap, e - 20), np.ldexp(Ap, e + 20)
    bl = np.ldexp(b, e - 20)
    say("split range: factorisations")
    dA = dev(O.stage(K, low))
    _, dinfo = P.getrf_ozaki(K, s, dA)
    assert int(host(dinfo)[0]) == -3
    LUo, ipo, info_o = O.getrf_ozaki(K, O.stage(K, ok), s)
    dA = dev(O.stage(K, ok))
    dip, dinfo = P.getrf_ozaki(K, s, dA)
    assert int(host(dinfo)[0]) == info_o == 0
    np.testing.assert_array_equal(host(dip), ipo)
    np.testing.assert_array_equal(host(dA), LUo)
    say("split range: refinement")
    ref = O.refine(low, bl, K, ozaki=s)
    out = P.refine(dev(low), dev(bl), K, ozaki=s)
    assert out["status"] == ref["status"] == O.CONVERGED and out["iters"] == ref["iters"]
    np.testing.assert_array_equal(host(out["x"]), ref["x"])
    say("split range: asynchronous refinement")
    x = torch.empty((4, n), dtype=torch.float64, device="cuda")
    res = torch.zeros(P.refine_result_bytes(), dtype=torch.uint8, device="cuda")
    work = torch.empty(P.refine_workspace_size(n, K), dtype=torch.uint8, device="cuda")
    P.refine_async(dev(low), dev(bl), K, res, x, work, ozaki=s)
    r = P.refine_result(res)
    assert r["status"] == P.BNC_SPLIT_RANGE
    assert not host(x).any()
