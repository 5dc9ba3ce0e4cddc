"""Parity at the benchmark's full size (n = 4096, randsvd with condition
number 1e10, triple-double factor, quad-double refinement), in the launch
configuration the benchmark times.  The oracle cannot factor n = 4096 in
test time, so the checks are properties that hold at any size:
  * the refined solution matches the exact solution (all ones; the
    right-hand side is exact in quad-double) to 1e-60, for the K-word and
    the split (Ozaki) factorisations;
  * sampled entries of P A - L U, computed exactly by the oracle from the
    GPU factor's words, are within the factor's backward-error bound.
"""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from helpers import dev, host

pytestmark = pytest.mark.gpu

N = 4096


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
def problem():
    say("generating randsvd n", N)
    Ap, b, exact = synth.problem("randsvd", N, config=2, instance=0, cond=1e10)
    assert exact
    return Ap, b


def max_err_vs_ones(x):
    return float(np.max(np.abs((x[0] - 1.0) + x[1] + x[2] + x[3])))


@pytest.mark.parametrize("oz", [0, 5, 8])
def test_fullsize_refine_reaches_quad_double(P, problem, oz):
    Ap, b = problem
    say("refine n", N, "ozaki", oz)
    out = P.refine(dev(Ap), dev(b), 3, ozaki=oz)
    assert out["status"] == P.BNC_CONVERGED
    assert not out["residual_inexact"]
    assert max_err_vs_ones(host(out["x"])) <= 1e-60


def permuted_rows(ipiv, n):
    perm = np.arange(n)
    for k, p in enumerate(ipiv):
        perm[k], perm[p] = perm[p], perm[k]
    return perm


@pytest.mark.parametrize("oz", [0, 5, 8])
def test_fullsize_factor_backward_error_sampled(P, problem, oz):
    Ap, _ = problem
    K = 3
    A = O.stage(K, Ap)
    dA = dev(A)
    say("getrf n", N, "ozaki", oz)
    if oz:
        dipiv, dinfo = P.getrf_ozaki(K, oz, dA)
    else:
        dipiv, dinfo = P.getrf(K, dA)
    assert int(host(dinfo)[0]) == 0
    LU = host(dA)
    ipiv = host(dipiv)
    assert np.all(ipiv >= np.arange(N)) and np.all(ipiv < N)
    perm = permuted_rows(ipiv, N)
    # partial pivoting bounds every multiplier by one
    assert np.abs(np.tril(LU[0].T, -1)).max() <= 1.0
    g = np.random.default_rng(5)
    pts = [(0, 0), (N - 1, N - 1), (N - 1, 0), (0, N - 1), (2000, 2100), (4000, 63), (64, 4000)]
    pts += [tuple(int(v) for v in g.integers(0, N, 2)) for _ in range(9)]
    u = 2.0 ** (-53 * K)
    for i, j in pts:
        m = min(i, j)
        # words of L(i, 0..m) (unit diagonal when m == i) and U(0..m, j)
        Lw = LU[:, :m + 1, i].copy()
        if m == i:
            Lw[:, i] = [1.0, 0.0, 0.0]
        Uw = LU[:, j, :m + 1]
        p = np.repeat(Lw, K, axis=0).ravel()          # word a of L times word c of U
        q = np.tile(Uw, (K, 1)).ravel()
        a_ij = A[:, j, perm[i]]
        pp = np.concatenate([p, a_ij])
        qq = np.concatenate([q, np.ones(K)])
        sg = np.concatenate([np.ones(p.size, np.int32), -np.ones(K, np.int32)])
        r, bad = O.exact_round(4, pp, qq, sg)
        assert not bad
        scale = float(np.sum(np.abs(Lw[0]) * np.abs(Uw[0])))
        bound = 16 * (m + 1) * u * scale
        if oz:  # dropped slice pairs, relative to the row and column scales
            bound += 64 * (oz + 2) * 2.0 ** (-20 * oz) * (m + 1) * np.abs(Lw[0]).max() * np.abs(Uw[0]).max()
        assert abs(r[0]) <= bound + 1e-300, (i, j, r[0], bound)


@pytest.mark.parametrize("oz", [0, 5])
def test_beyond_one_panel_workgroup_per_64_rows(P, oz):
    """n = 4160: the first panels have 65 workgroups and the substitutions 65
    blocks, one more than at n = 4096, with a 64-row tail everywhere; the
    refined solution must still reach 1e-60."""
    n = 4160
    say("generating randsvd n", n)
    Ap, b, exact = synth.problem("randsvd", n, config=2, instance=1, cond=1e8)
    assert exact
    say("refine n", n, "ozaki", oz)
    out = P.refine(dev(Ap), dev(b), 3, ozaki=oz)
    assert out["status"] == P.BNC_CONVERGED and out["info"] == 0
    assert max_err_vs_ones(host(out["x"])) <= 1e-60
