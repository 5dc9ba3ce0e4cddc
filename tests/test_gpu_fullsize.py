"""Parity at the benchmark's scale and forms.

n = 2048 (32 panel workgroups, 31 look-ahead steps), bit for bit against
the oracle: pivots, info and every word of the factor, and the refined
solution, correction count and status, for the headline form (double-double
factor, split trailing update with 5 slices), the 4-slice split form, the
plain triple-double form, and quad-double-word entries at condition 1e25
with a 7-slice triple-double factor.

n = 4096 (the benchmark's order and launch configuration): pivots and
every word of the 5- and 4-slice double-double split factors (the
benchmark's headline is the faster) against the oracle, bit for bit;
refinement to 1e-60 of the exact solution (all ones, exact in quad-double)
for every form the benchmark times, at condition 1e10 and (quad-double-word
entries) 1e25; and sampled entries of P A - L U, formed exactly by the
oracle from the GPU factor's words, within the factor's backward-error
bound (the split form's bound from its slice width beta(K, S)).
"""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from helpers import dev, host

pytestmark = pytest.mark.gpu

N = 4096
N2 = 2048


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


@pytest.fixture(scope="module")
def problem():
    say("generating randsvd n", N)
    Ap, b, exact = synth.problem("randsvd", N, config=2, instance=0, cond=1e10)
    assert exact
    return Ap, b


@pytest.fixture(scope="module")
def problem_words():
    say("generating quad-double-word randsvd n", N, "cond 1e25")
    Ap, b, exact = synth.problem("randsvd_words", N, config=2, instance=0, cond=1e25)
    assert exact and Ap.shape[0] == 4
    return Ap, b


@pytest.fixture(scope="module")
def problem2():
    say("generating randsvd n", N2)
    Ap, b, exact = synth.problem("randsvd", N2, config=1, instance=0, cond=1e10)
    assert exact
    return Ap, b


def max_err_vs_ones(x):
    return float(np.max(np.abs((x[0] - 1.0) + x[1] + x[2] + x[3])))


def factor_gpu(P, K, oz, A):
    dA = dev(A)
    if oz:
        dipiv, dinfo = P.getrf_ozaki(K, oz, dA)
    else:
        dipiv, dinfo = P.getrf(K, dA)
    return host(dA), host(dipiv), int(host(dinfo)[0])


# ---- n = 2048, bit for bit ----------------------------------------------

FORMS2 = [(2, 5), (2, 4), (3, 0)]


@pytest.mark.parametrize("K,oz", FORMS2)
def test_n2048_factor_and_refine_bitexact(P, problem2, K, oz):
    Ap, b = problem2
    say("oracle refine n", N2, "K", K, "ozaki", oz)
    ref = O.refine(Ap, b, K, ozaki=oz)
    assert ref["status"] == O.CONVERGED and ref["info"] == 0
    say("gpu getrf n", N2, "K", K, "ozaki", oz)
    LU, ipiv, info = factor_gpu(P, K, oz, O.stage(K, Ap))
    assert info == 0
    np.testing.assert_array_equal(ipiv, ref["ipiv"])
    np.testing.assert_array_equal(LU, ref["LU"])
    say("gpu refine n", N2, "K", K, "ozaki", oz)
    out = P.refine(dev(Ap), dev(b), K, ozaki=oz)
    assert out["status"] == ref["status"] and out["iters"] == ref["iters"]
    np.testing.assert_array_equal(host(out["x"]), ref["x"])
    assert max_err_vs_ones(ref["x"]) <= 1e-60


def test_n2048_quad_double_words_cond_1e25_bitexact(P):
    say("generating quad-double-word randsvd n", N2, "cond 1e25")
    Ap, b, exact = synth.problem("randsvd_words", N2, config=1, instance=1, cond=1e25)
    assert exact and Ap.shape[0] == 4
    K, oz = 3, 7
    say("oracle refine words K", K, "ozaki", oz)
    ref = O.refine(Ap, b, K, ozaki=oz)
    assert ref["status"] == O.CONVERGED
    say("gpu getrf words")
    LU, ipiv, info = factor_gpu(P, K, oz, O.stage(K, Ap))
    assert info == 0
    np.testing.assert_array_equal(ipiv, ref["ipiv"])
    np.testing.assert_array_equal(LU, ref["LU"])
    say("gpu refine words")
    out = P.refine(dev(Ap), dev(b), K, ozaki=oz)
    assert out["status"] == ref["status"] and out["iters"] == ref["iters"]
    np.testing.assert_array_equal(host(out["x"]), ref["x"])
    assert max_err_vs_ones(ref["x"]) <= 1e-60


# ---- n = 4096 --------------------------------------------------------------

@pytest.mark.timeout(1200)
@pytest.mark.parametrize("K,oz", [(2, 5), (2, 4)])
def test_n4096_headline_factor_bitexact(P, problem, K, oz):
    """The split double-double forms the benchmark times (5 and 4 slices,
    the faster of which is its headline), factorised at the benchmark's
    order: every pivot and every word equal to the oracle's blocked split
    LU."""
    Ap, _ = problem
    A = O.stage(K, Ap)
    say("gpu getrf n", N, "K", K, "ozaki", oz)
    LU, ipiv, info = factor_gpu(P, K, oz, A)
    assert info == 0
    say("oracle getrf n", N, "K", K, "ozaki", oz, "threads", O.threads())
    LUo, ipo, info_o = O.getrf_ozaki(K, A, oz)
    assert info_o == 0
    np.testing.assert_array_equal(ipiv, ipo)
    np.testing.assert_array_equal(LU, LUo)


@pytest.mark.parametrize("K,oz", [(3, 0), (2, 5), (2, 4), (3, 5), (3, 8)])
def test_fullsize_refine_reaches_quad_double(P, problem, K, oz):
    Ap, b = problem
    say("refine n", N, "K", K, "ozaki", oz)
    out = P.refine(dev(Ap), dev(b), K, ozaki=oz)
    assert out["status"] == P.BNC_CONVERGED
    assert not out["residual_inexact"]
    assert max_err_vs_ones(host(out["x"])) <= 1e-60


@pytest.mark.parametrize("K,oz", [(3, 0), (3, 7), (2, 7)])
def test_fullsize_cond_1e25_quad_double_words(P, problem_words, K, oz):
    Ap, b = problem_words
    say("refine words n", N, "K", K, "ozaki", oz)
    out = P.refine(dev(Ap), dev(b), K, ozaki=oz)
    assert out["status"] == P.BNC_CONVERGED
    assert not out["residual_inexact"]
    assert max_err_vs_ones(host(out["x"])) <= 1e-60


def permuted_rows(ipiv, n):
    perm = np.arange(n)
    for k, p in enumerate(ipiv):
        perm[k], perm[p] = perm[p], perm[k]
    return perm


@pytest.mark.parametrize("K,oz", [(3, 0), (2, 5), (2, 4), (3, 5), (3, 8)])
def test_fullsize_factor_backward_error_sampled(P, problem, K, oz):
    Ap, _ = problem
    A = O.stage(K, Ap)
    say("getrf n", N, "K", K, "ozaki", oz)
    LU, ipiv, info = factor_gpu(P, K, oz, A)
    assert info == 0
    assert np.all(ipiv >= np.arange(N)) and np.all(ipiv < N)
    perm = permuted_rows(ipiv, N)
    # partial pivoting bounds every multiplier by one
    assert np.abs(np.tril(LU[0].T, -1)).max() <= 1.0
    g = np.random.default_rng(5)
    pts = [(0, 0), (N - 1, N - 1), (N - 1, 0), (0, N - 1), (2000, 2100), (4000, 63), (64, 4000)]
    pts += [tuple(int(v) for v in g.integers(0, N, 2)) for _ in range(9)]
    u = 2.0 ** (-53 * K)
    beta = O.oz_beta(K, oz) if oz else 0
    for i, j in pts:
        m = min(i, j)
        # words of L(i, 0..m) (unit diagonal when m == i) and U(0..m, j)
        Lw = LU[:, :m + 1, i].copy()
        if m == i:
            Lw[:, i] = [1.0] + [0.0] * (K - 1)
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
        if oz:  # dropped slice pairs: below 2^-(beta oz) of the row and column scales per product, a few per pair
            bound += 64 * (oz + 2) * 2.0 ** (-beta * oz) * (m + 1) * np.abs(Lw[0]).max() * np.abs(Uw[0]).max()
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
