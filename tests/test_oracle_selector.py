"""Pins for the oracle's features and MLP (the learned precision choice,
a project addition on top of the paper's refinement loop, Sec. 2).

Features: closed forms on diagonal, symmetric and singular matrices; the
LU-derived features against LAPACK's factors (scipy); Hager's estimate is
exact for diagonal matrices and otherwise a lower bound of ||A^-1||_1 that
never decreases from step to step (Hager 1984; Higham 1988).
MLP: back-propagated gradients against central finite differences in
float64; Adam's first step moves every parameter by -lr g / (|g| + eps).
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import oracle.selector as S
import synth


def planes(A):
    return synth.planes(np.asarray(A, dtype=np.float64))


def rhs(Ap):
    b, _ = synth.rhs_ones(Ap)
    return b


def test_diagonal_matrix_closed_forms():
    d = np.array([1.0, 0.5, 2.0 ** -20, 4.0, 2.0 ** -7])
    A = np.diag(d)
    Ap = planes(A)
    f = S.features(Ap, rhs(Ap))
    n = len(d)
    assert f[0] == math.log2(n)
    assert f[1] == pytest.approx(0.5 * math.log2(np.sum(d * d)), abs=1e-12)
    assert f[5] == 100.0 and f[7] == 1.0          # every row dominant (no off-diagonal mass)
    assert f[11] == -1100.0                       # symmetric
    assert f[13] == pytest.approx(math.log2(d.min() / d.max()), abs=1e-12)
    # Hager on a diagonal matrix: the first step gives ||A^-1 (e/n)||_1 =
    # mean(1/d); the second picks e_j at the smallest d and is exact,
    # ||A||_1 ||A^-1||_1 = max d / min d, and there ||z||_inf = z^T x stops it
    assert f[17] == pytest.approx(math.log2(d.max() * np.mean(1.0 / d)), abs=1e-12)
    for q in (18, 19):
        assert f[q] == pytest.approx(math.log2(d.max() / d.min()), abs=1e-12)
    assert f[22] == 2.0
    assert f[21] == -1100.0                       # binary64 solve exact, zero residual


def test_symmetric_and_singular():
    g = np.random.default_rng(3)
    M = g.uniform(-1, 1, (12, 12))
    Ap = planes(M + M.T)
    f = S.features(Ap, rhs(Ap))
    assert f[11] == -1100.0
    Z = g.uniform(-1, 1, (10, 10))
    Z[:, 4] = 0.0
    Ap = planes(Z)
    f = S.features(Ap, rhs(Ap))
    norm1 = np.abs(Z).sum(axis=0).max()
    assert f[17] == f[18] == f[19] == pytest.approx(1000 + math.log2(norm1), abs=1e-12)
    assert f[20] == 1100.0 and f[22] == 0.0


@pytest.mark.parametrize("kind,cond", [("uniform", 0), ("randsvd", 1e6), ("randsvd", 1e14)])
def test_lu_features_match_lapack_and_hager_is_a_lower_bound(kind, cond):
    for inst in range(4):
        n = 30 + 17 * inst
        Ap, b, _ = synth.problem(kind, n, config=3, instance=inst, cond=cond or 1e3)
        A = Ap[0].T
        f = S.features(Ap, b)
        lu, piv = sla.lu_factor(A)
        U = np.triu(lu)
        ud = np.abs(np.diag(U))
        # the smallest pivot is determined to about kappa n u relative
        tol = 2.0 * (cond or 1e3) * n * 2.0 ** -52 + 1e-9
        assert f[13] == pytest.approx(math.log2(ud.min() / ud.max()), abs=tol)
        assert f[12] == pytest.approx(math.log2(np.abs(U).max() / np.abs(A).max()), abs=1e-9)
        inv1 = np.abs(np.linalg.inv(A)).sum(axis=0).max()
        norm1 = np.abs(A).sum(axis=0).max()
        true = math.log2(norm1 * inv1)
        # (the reference inverse and the estimate's solves carry kappa n u)
        assert f[17] <= f[18] <= f[19] <= true + math.log2(1.0 + tol)
        assert f[19] >= true - math.log2(3 * n)   # within the usual small factor
        # backward error of the binary64 solve is of order n u
        assert f[21] <= math.log2(n * 2.0 ** -50)


def test_mlp_gradient_matches_finite_differences():
    g = np.random.default_rng(11)
    P = g.normal(0, 0.3, S.NPARAM)
    B = 7
    X = g.normal(0, 1, (B, S.MI))
    norm = np.concatenate([g.normal(0, 0.1, S.MI), 1.0 + 0.1 * g.random(S.MI)])
    cls = g.integers(0, 4, B)
    tgt = g.normal(1.5, 1.0, B)
    loss, G = S.loss_and_grad(P, X, norm, cls, tgt)
    idx = np.concatenate([g.choice(S.NPARAM, 60, replace=False), [S.NPARAM - 1, S.NPARAM - 5, 0]])
    h = 1e-6
    for i in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[i] += h
        Pm[i] -= h
        fd = (S.loss_and_grad(Pp, X, norm, cls, tgt)[0] - S.loss_and_grad(Pm, X, norm, cls, tgt)[0]) / (2 * h)
        assert abs(fd - G[i]) <= 1e-6 * max(1.0, abs(G[i])), i


def test_adam_first_step_is_lr_times_sign():
    g = np.random.default_rng(12)
    P = g.normal(0, 1, 50)
    G = g.normal(0, 1, 50)
    P1, M, V = S.adam(P, G, np.zeros(50), np.zeros(50), 1, lr=1e-2)
    # bias-corrected m = g and v = g^2: the step is -lr g / (|g| + eps)
    np.testing.assert_allclose(P1 - P, -1e-2 * G / (np.abs(G) + 1e-8), rtol=1e-9)
    np.testing.assert_allclose(M, 0.1 * G)
    np.testing.assert_allclose(V, 0.001 * G * G)
