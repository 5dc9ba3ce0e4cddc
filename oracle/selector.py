"""ORACLE -- test infrastructure: plain definitions of the learned
precision choice's numbers (the project's addition on top of the paper's
refinement loop, Kouya 2021 Sec. 2 / Listing 1).

  * features(): the 24 binary64 features of one system, in the order and
    with the operation sequence the library documents (sums in index
    order, the binary64 LU and substitutions of the oracle's getrf/getrs
    with K = 1, Hager's 1-norm estimate: Hager, SIAM J. Sci. Stat. Comput.
    5 (1984); Higham, ACM TOMS 14 (1988)).
  * MLP 24 -> 64 -> 64 -> 5 with ReLU, its loss (cross-entropy of the
    first 4 outputs + 0.5 Huber of the 5th), gradients by hand-derived
    back-propagation, and Adam (Kingma and Ba 2015) -- all in float64.
Only tests/ may import this module.
"""
from __future__ import annotations

import math

import numpy as np

from . import fms, getrf, getrs, mul, recip

NFEAT = 24
MI, MH, MO, MC = 24, 64, 5, 4
HUBER_W = 0.5
LG_CAP = 1100.0


def lg(x: float) -> float:
    if not x > 0.0:
        return -LG_CAP
    v = math.log2(x)
    return max(-LG_CAP, min(LG_CAP, v))


def seq_sum(v) -> float:
    """Sum in index order (left to right, one rounding per addition)."""
    v = np.asarray(v, dtype=np.float64).ravel()
    return float(np.cumsum(v)[-1]) if v.size else 0.0


def _solve(LU, ipiv, y):
    """A^-1 y with the oracle's K = 1 substitutions."""
    return getrs(1, LU, ipiv, np.asarray(y, dtype=np.float64)[None, :])[0]


def _solve_t(LU, ipiv, c):
    """A^-T c: U^T w = c (w_k = w_k (1/u_kk), then w_i -= u_ki w_k for
    i > k), L^T v = w (v_i -= l_ki v_k for i < k, decreasing k), then the
    row swaps undone in reverse order."""
    M = LU[0].T  # M[i, j] = entry (i, j)
    n = M.shape[0]
    w = np.array(c, dtype=np.float64)
    for k in range(n):
        w[k] = mul(1, w[k:k + 1][None, :], recip(1, M[k:k + 1, k][None, :]))[0, 0]
        if k + 1 < n:
            w[k + 1:] = fms(1, w[k + 1:][None, :], M[k, k + 1:][None, :], np.full((1, n - k - 1), w[k]))[0]
    for k in range(n - 1, 0, -1):
        w[:k] = fms(1, w[:k][None, :], M[k, :k][None, :], np.full((1, k), w[k]))[0]
    for k in range(n - 1, -1, -1):
        p = int(ipiv[k])
        if p != k:
            w[k], w[p] = w[p], w[k]
    return w


def features(Ap: np.ndarray, b: np.ndarray) -> np.ndarray:
    """24 features (float64, before rounding to binary32) of the system with
    binary64 matrix Ap (1, n, n) K-plane and right-hand side b (4, n)."""
    n = Ap.shape[1]
    A = Ap[0].T  # A[i, j] = entry (i, j)
    f = np.zeros(NFEAT)
    absA = np.abs(A)
    rowabs = np.array([seq_sum(absA[i]) for i in range(n)])
    rowsq = np.array([seq_sum(A[i] * A[i]) for i in range(n)])
    off = np.array([seq_sum(np.delete(absA[i], i)) for i in range(n)])
    colabs = np.array([seq_sum(absA[:, j]) for j in range(n)])
    colsq = np.array([seq_sum(A[:, j] * A[:, j]) for j in range(n)])
    symsq = np.array([seq_sum((A[:, j] - A[j, :]) * (A[:, j] - A[j, :])) for j in range(n)])
    diag = np.abs(np.diag(A))
    ratio = np.where(off > 0.0, diag / np.where(off > 0.0, off, 1.0), 2.0 ** 100)
    fro2 = seq_sum(colsq)
    sym2 = seq_sum(symsq)
    dg2 = seq_sum(diag * diag)
    rsum = seq_sum(ratio)
    ndom = seq_sum((ratio > 1.0).astype(np.float64))
    norm1, norminf, amax = colabs.max(), rowabs.max(), absA.max()
    fro = math.sqrt(fro2)
    lfro = lg(fro)
    f[0] = lg(float(n))
    f[1] = lfro
    f[2] = lg(norm1) - lfro
    f[3] = lg(norminf) - lfro
    f[4] = lg(amax) - lfro
    f[5] = lg(ratio.min())
    f[6] = lg(rsum / n)
    f[7] = ndom / n
    f[8] = 0.5 * lg(dg2) - lfro
    f[9] = 0.5 * (lg(colsq.min()) - lg(colsq.max()))
    f[10] = 0.5 * (lg(rowsq.min()) - lg(rowsq.max()))
    f[11] = lg(math.sqrt(sym2) / fro) if fro > 0.0 else -LG_CAP

    LU, ipiv, info = getrf(1, Ap)
    M = LU[0].T
    umax = np.abs(np.triu(M)).max()
    ud = np.abs(np.diag(M))
    udmax, udmin = ud.max(), ud.min()
    lgs = seq_sum([lg(v) for v in ud])
    f[12] = lg(umax) - lg(amax)
    f[13] = lg(udmin) - lg(udmax)
    f[14] = lg(udmax) - lfro
    f[15] = lgs / n - lg(udmax)
    f[16] = float(np.count_nonzero(ud < 2.0 ** -26 * udmax)) / n

    est = [2.0 ** 1000] * 3
    steps = 0
    if info:
        f[20] = LG_CAP
        f[21] = 0.0
    else:
        x = np.full(n, 1.0 / n)
        jprev = -1
        for it in range(3):
            y = _solve(LU, ipiv, x)
            g = seq_sum(np.abs(y))
            steps = it + 1
            for q in range(it, 3):
                est[q] = g
            xi = np.where(y < 0.0, -1.0, 1.0)
            z = _solve_t(LU, ipiv, xi)
            az = np.abs(z)
            j = int(np.argmax(az))  # first index of the maximum
            zx = seq_sum(z * x) if jprev < 0 else z[jprev]
            if az[j] <= zx:
                break
            jprev = j
            x = np.zeros(n)
            x[j] = 1.0
        b0 = b[0].copy()
        x0 = _solve(LU, ipiv, b0)
        r = np.array([seq_sum(np.concatenate([[b0[i]], -(A[i] * x0)])) for i in range(n)])
        xmax = np.abs(x0).max()
        f[20] = lg(xmax) - lg(np.abs(b0).max()) + lg(norminf)
        f[21] = lg(np.abs(r).max()) - lg(norminf) - lg(xmax)
    f[17:20] = [lg(norm1) + lg(e) for e in est]
    f[22] = float(steps)
    f[23] = lg(diag.max()) - lg(amax)
    return np.clip(f, -LG_CAP, LG_CAP)


# --------------------------------------------------------------------------
# MLP
# --------------------------------------------------------------------------

def unpack(P):
    P = np.asarray(P, dtype=np.float64)
    o = 0
    W1 = P[o:o + MI * MH].reshape(MI, MH); o += MI * MH
    b1 = P[o:o + MH]; o += MH
    W2 = P[o:o + MH * MH].reshape(MH, MH); o += MH * MH
    b2 = P[o:o + MH]; o += MH
    W3 = P[o:o + MH * MO].reshape(MH, MO); o += MH * MO
    b3 = P[o:o + MO]; o += MO
    return W1, b1, W2, b2, W3, b3


NPARAM = MI * MH + MH + MH * MH + MH + MH * MO + MO


def forward(P, X, norm):
    W1, b1, W2, b2, W3, b3 = unpack(P)
    norm = np.asarray(norm, dtype=np.float64)
    Xn = (np.asarray(X, dtype=np.float64) - norm[:MI]) * norm[MI:]
    H1 = np.maximum(Xn @ W1 + b1, 0.0)
    H2 = np.maximum(H1 @ W2 + b2, 0.0)
    return Xn, H1, H2, H2 @ W3 + b3


def loss_and_grad(P, X, norm, cls, tgt):
    """Mean over the batch of CE(softmax(o[:4]), cls) + 0.5 Huber(o[4] - tgt)
    and its gradient with respect to the packed parameters."""
    W1, b1, W2, b2, W3, b3 = unpack(P)
    Xn, H1, H2, O = forward(P, X, norm)
    B = Xn.shape[0]
    cls = np.asarray(cls)
    logits = O[:, :MC]
    m = logits.max(axis=1, keepdims=True)
    e = np.exp(logits - m)
    z = e.sum(axis=1, keepdims=True)
    ce = (np.log(z[:, 0]) + m[:, 0] - logits[np.arange(B), cls])
    d = O[:, MC] - np.asarray(tgt, dtype=np.float64)
    ad = np.abs(d)
    hub = np.where(ad <= 1.0, 0.5 * d * d, ad - 0.5)
    loss = float(np.mean(ce + HUBER_W * hub))
    dO = np.zeros_like(O)
    dO[:, :MC] = e / z
    dO[np.arange(B), cls] -= 1.0
    dO[:, MC] = HUBER_W * np.where(ad <= 1.0, d, np.sign(d))
    dO /= B
    dW3 = H2.T @ dO
    db3 = dO.sum(axis=0)
    D2 = (dO @ W3.T) * (H2 > 0.0)
    dW2 = H1.T @ D2
    db2 = D2.sum(axis=0)
    D1 = (D2 @ W2.T) * (H1 > 0.0)
    dW1 = Xn.T @ D1
    db1 = D1.sum(axis=0)
    G = np.concatenate([dW1.ravel(), db1, dW2.ravel(), db2, dW3.ravel(), db3])
    return loss, G


def adam(P, G, M, V, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    M = b1 * M + (1.0 - b1) * G
    V = b2 * V + (1.0 - b2) * G * G
    P = P - lr * (M / (1.0 - b1 ** step)) / (np.sqrt(V / (1.0 - b2 ** step)) + eps)
    return P, M, V
