"""GPU parity: the HIP path (through the C-ABI) against the oracle, bit for
bit, on seeded inputs spanning several tiles and ragged tails.

The device arithmetic, the blocked factorisation, the blocked substitutions
and the exact residual all follow the same fixed operation order as the
oracle's plain loops, so every word and every pivot must be identical.
"""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from helpers import dev, host, rand_words

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


@pytest.mark.parametrize("K", [1, 2, 3, 4])
def test_primitives_bitexact(P, K):
    g = np.random.default_rng(900 + K)
    n = 3000
    a, b, c = rand_words(g, K, n), rand_words(g, K, n), rand_words(g, K, n)
    ab = O.mul(K, a, b)
    c[:, :1000] = ab[:, :1000]
    c[0, :1000] *= 1 + 2.0 ** -40
    say("primitives K", K)
    da, db, dc = dev(a), dev(b), dev(c)
    np.testing.assert_array_equal(host(P.mw_apply(P.OP_FMS, K, da, db, dc)), O.fms(K, c, a, b))
    np.testing.assert_array_equal(host(P.mw_apply(P.OP_MUL, K, da, db)), O.mul(K, a, b))
    np.testing.assert_array_equal(host(P.mw_apply(P.OP_ADD, K, da, db)), O.add(K, a, b))
    np.testing.assert_array_equal(host(P.mw_apply(P.OP_RECIP, K, da)), O.recip(K, a))
    q = rand_words(g, 4, n)
    np.testing.assert_array_equal(host(P.mw_apply(P.OP_ROUND4, K, dev(q))), O.round_words(K, q))


CASES = [(1, 1), (2, 5), (3, 63), (4, 64), (1, 65), (2, 130), (3, 200), (4, 129), (3, 257), (2, 300)]


@pytest.mark.parametrize("K,n", CASES)
def test_getrf_getrs_bitexact(P, K, n):
    Ap, b, _ = synth.problem("uniform", n, config=0, instance=100 + n)
    A = O.stage(K, Ap)
    LU, ipiv, info = O.getrf(K, A)
    say("getrf K", K, "n", n)
    dA = dev(A)
    dipiv, dinfo = P.getrf(K, dA)
    np.testing.assert_array_equal(host(dipiv), ipiv)
    assert int(host(dinfo)[0]) == info == 0
    np.testing.assert_array_equal(host(dA), LU)
    bf = O.round_words(K, b)
    x = O.getrs(K, LU, ipiv, bf)
    say("getrs K", K, "n", n)
    dx = dev(bf)
    P.getrs(K, dA, dipiv, dx)
    np.testing.assert_array_equal(host(dx), x)
    # several right-hand sides at once
    B = np.stack([bf, 0.5 * bf, -bf], axis=1)
    X = O.getrs(K, LU, ipiv, B)
    dB = dev(B)
    P.getrs(K, dA, dipiv, dB)
    np.testing.assert_array_equal(host(dB), X)


@pytest.mark.parametrize("K,n", [(2, 300), (3, 257), (1, 64)])
def test_getrs_any_swap_sequence_bitexact(P, K, n):
    """Substitutions with a pivot sequence that no factorisation produced
    (random targets, repeats, no-op swaps) follow the oracle bit for bit;
    entries outside [k, n) act as no interchange."""
    import torch
    g = np.random.default_rng(4400 + n)
    Ap, b, _ = synth.problem("uniform", n, config=0, instance=300 + n)
    LU, _, info = O.getrf(K, O.stage(K, Ap))
    assert info == 0
    ipiv = np.array([g.integers(k, n) for k in range(n)], dtype=np.int64)
    ipiv[::7] = np.arange(n)[::7]
    ipiv[n // 2:n // 2 + 5] = n - 1
    bf = O.round_words(K, b)
    say("getrs any ipiv K", K, "n", n)
    dLU, dx = dev(LU), dev(bf)
    P.getrs(K, dLU, torch.from_numpy(ipiv).cuda(), dx)
    np.testing.assert_array_equal(host(dx), O.getrs(K, LU, ipiv, bf))
    bad = ipiv.copy()
    idx = np.arange(3, n, 11)
    bad[idx] = np.where(idx % 2 == 0, -1, n + 5)
    bad[5] = 2
    noop = ipiv.copy()
    noop[idx] = idx
    noop[5] = 5
    dy, dz = dev(bf), dev(bf)
    P.getrs(K, dLU, torch.from_numpy(bad).cuda(), dy)
    P.getrs(K, dLU, torch.from_numpy(noop).cuda(), dz)
    np.testing.assert_array_equal(host(dy), host(dz))
    np.testing.assert_array_equal(host(dz), O.getrs(K, LU, noop, bf))


@pytest.mark.parametrize("K", [1, 3])
def test_getrf_randsvd_illconditioned_bitexact(P, K):
    n = 160
    Ap, b, _ = synth.problem("randsvd", n, config=1, instance=1, cond=1e15)
    A = O.stage(K, Ap)
    LU, ipiv, info = O.getrf(K, A)
    say("getrf randsvd K", K)
    dA = dev(A)
    dipiv, dinfo = P.getrf(K, dA)
    np.testing.assert_array_equal(host(dipiv), ipiv)
    np.testing.assert_array_equal(host(dA), LU)


def test_getrf_singular_and_constructed(P):
    # exact zero pivot at the last step; LAPACK info convention
    A = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [1.0, 0.0, 1.0]])
    for K in (1, 2, 3, 4):
        Pl = np.zeros((K, 3, 3))
        Pl[0] = A.T
        say("singular K", K)
        dA = dev(Pl)
        dipiv, dinfo = P.getrf(K, dA)
        LU, ipiv, info = O.getrf(K, Pl)
        assert int(host(dinfo)[0]) == info == 3
        np.testing.assert_array_equal(host(dipiv), ipiv)
        np.testing.assert_array_equal(host(dA), LU)
    # zero first column
    Z = np.zeros((70, 70))
    Z[:, 1:] = np.random.default_rng(3).uniform(-1, 1, (70, 69))
    Pl = np.zeros((2, 70, 70))
    Pl[0] = Z.T
    say("zero column")
    dA = dev(Pl)
    dipiv, dinfo = P.getrf(2, dA)
    LU, ipiv, info = O.getrf(2, Pl)
    assert int(host(dinfo)[0]) == info == 1
    np.testing.assert_array_equal(host(dipiv), ipiv)
    np.testing.assert_array_equal(host(dA), LU)


def test_ties_take_first_row(P):
    """Integer matrix with many equal magnitudes in every column."""
    g = np.random.default_rng(5)
    n = 96
    A = g.choice([-2.0, -1.0, 1.0, 2.0], size=(n, n))
    for K in (1, 3):
        Pl = np.zeros((K, n, n))
        Pl[0] = A.T
        LU, ipiv, info = O.getrf(K, Pl)
        say("ties K", K)
        dA = dev(Pl)
        dipiv, dinfo = P.getrf(K, dA)
        np.testing.assert_array_equal(host(dipiv), ipiv)
        np.testing.assert_array_equal(host(dA), LU)


@pytest.mark.parametrize("aw,n", [(1, 1), (1, 7), (1, 64), (1, 300), (4, 5), (4, 130)])
def test_residual_bitexact(P, aw, n):
    g = np.random.default_rng(70 + n + aw)
    A = np.zeros((aw, n, n))
    flat = rand_words(g, aw, n * n, spread=2)
    A[:] = flat.reshape(aw, n, n)
    x = rand_words(g, 4, n, spread=1)
    b = rand_words(g, 4, n, spread=1)
    r = O.residual(A, x, b)
    say("residual aw", aw, "n", n)
    dr, flag = P.residual(dev(A), dev(x), dev(b))
    assert int(host(flag)[0]) == 0
    np.testing.assert_array_equal(host(dr), r)


def test_residual_near_solution_bitexact(P):
    """Residual of a nearly converged x: heavy cancellation, tiny result."""
    n = 256
    Ap, b, exact = synth.problem("randsvd", n, config=1, instance=2, cond=1e10)
    res = O.refine(Ap, b, 3, max_iter=2)
    x = res["x"]
    r = O.residual(Ap, x, b)
    say("residual near solution")
    dr, flag = P.residual(dev(Ap), dev(x), dev(b))
    assert int(host(flag)[0]) == 0
    np.testing.assert_array_equal(host(dr), r)


@pytest.mark.parametrize("K,n,kind,cond", [(2, 128, "uniform", 0), (3, 128, "uniform", 0), (4, 70, "uniform", 0),
                                           (1, 100, "uniform", 0), (2, 200, "randsvd", 1e10),
                                           (3, 200, "randsvd", 1e15)])
def test_refine_bitexact(P, K, n, kind, cond):
    Ap, b, exact = synth.problem(kind, n, config=0 if kind == "uniform" else 1, instance=3, cond=cond or 1e3)
    ref = O.refine(Ap, b, K)
    say("refine K", K, "n", n, kind)
    out = P.refine(dev(Ap), dev(b), K)
    x = host(out["x"])
    assert out["status"] == ref["status"] == O.CONVERGED
    assert out["iters"] == ref["iters"]
    assert not out["residual_inexact"]
    np.testing.assert_array_equal(x, ref["x"])
    if exact:
        from oracle.exact import value
        err = max(float(abs(value(x[:, i]) - 1)) for i in range(n))
        assert err <= 1e-60


def test_refine_step_semantics_and_failures(P):
    n = 40
    Ap, b, _ = synth.problem("uniform", n, config=0, instance=9)
    for mi in (0, 1, 2):
        ref = O.refine(Ap, b, 2, max_iter=mi)
        say("refine max_iter", mi)
        out = P.refine(dev(Ap), dev(b), 2, max_iter=mi)
        assert out["iters"] == ref["iters"] and out["status"] == ref["status"]
        np.testing.assert_array_equal(host(out["x"]), ref["x"])
    A = np.array([[2.0, 1, 0, 1], [1, 3, 1, 0], [0, 1, 4, 1], [1, 3, 1, 0]])
    Ap = synth.planes(A)
    b, _ = synth.rhs_ones(Ap)
    say("refine singular")
    out = P.refine(dev(Ap), dev(b), 3)
    assert out["status"] == P.BNC_SINGULAR and out["info"] == O.refine(Ap, b, 3)["info"]
    Ap2 = Ap.copy()
    Ap2[0, 1, 1] = np.inf
    say("refine nonfinite")
    out = P.refine(dev(Ap2), dev(b), 3)
    assert out["status"] == P.BNC_NONFINITE
