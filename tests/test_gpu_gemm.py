"""GPU parity of the multi-word matrix multiply-subtract C <- C - A B
(Kouya 2021, Sec. 2 and Fig. 1: the library's block matrix multiplication;
the LU's trailing-update kernel exported through bnc_gemm_*) against the
oracle's plain triple loop, bit for bit: ragged shapes spanning several
tiles, the empty cases, and sampled entries of a large product."""
import sys

import numpy as np
import pytest

import oracle as O
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


def words(g, K, cols, rows, spread=4):
    if cols == 0 or rows == 0:
        return np.zeros((K, cols, rows))
    return np.stack([rand_words(g, K, rows, spread) for _ in range(cols)], axis=1)


@pytest.mark.parametrize("K", [1, 2, 3, 4])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (70, 33, 130), (129, 65, 64), (64, 200, 17), (5, 3, 0), (0, 4, 6)])
def test_gemm_bitexact(P, K, m, n, k):
    g = np.random.default_rng(1000 + 7 * K + m + 3 * n + 11 * k)
    A, B, C = words(g, K, k, m), words(g, K, n, k), words(g, K, n, m)
    say("gemm K", K, "m n k", m, n, k)
    want = O.gemm(K, A, B, C)
    dC = dev(C)
    P.gemm(K, dev(A), dev(B), dC)
    np.testing.assert_array_equal(host(dC), want)


def test_gemm_large_sampled(P):
    """m = n = 2048, k = 512, triple-double: 64 sampled entries, each
    computed by the oracle from its row of A and column of B alone."""
    K, m, n, k = 3, 2048, 2048, 512
    g = np.random.default_rng(4242)

    def big(cols, rows):  # word t on the scale 2^(-53 t): vectorised, need not be normalised
        return g.uniform(-1.0, 1.0, (K, cols, rows)) * np.exp2(-53.0 * np.arange(K))[:, None, None]

    A, B, C = big(k, m), big(n, k), big(n, m)
    say("gemm large", m, n, k)
    dC = dev(C)
    P.gemm(K, dev(A), dev(B), dC)
    got = host(dC)
    for t in range(64):
        i, j = int(g.integers(m)), int(g.integers(n))
        want = O.gemm(K, A[:, :, i:i + 1], B[:, j:j + 1, :], C[:, j:j + 1, i:i + 1])
        np.testing.assert_array_equal(got[:, j, i], want[:, 0, 0], err_msg=f"entry ({i}, {j})")


@pytest.mark.parametrize("K", [2, 3])
def test_gemm_padded_strides_through_the_abi(P, K):
    """Leading dimensions and plane strides larger than the matrices (views
    into bigger K-plane buffers), called through the C-ABI directly: the
    padding is left untouched and the product equals the oracle's."""
    import ctypes
    import torch
    m, n, k = 45, 37, 70
    lda, ldb, ldc = 53, 81, 64
    ldpa, ldpb, ldpc = lda * k + 11, ldb * n + 5, ldc * n + 7
    g = np.random.default_rng(77 + K)
    A, B, C = words(g, K, k, m), words(g, K, n, k), words(g, K, n, m)
    want = O.gemm(K, A, B, C)

    def pad(X, ld, ldp, fill):
        rows, cols = X.shape[2], X.shape[1]
        buf = np.full(K * ldp, fill)
        for w in range(K):
            for c in range(cols):
                buf[w * ldp + c * ld: w * ldp + c * ld + rows] = X[w, c]
        return buf

    bA, bB, bC = pad(A, lda, ldpa, 7.0), pad(B, ldb, ldpb, 9.0), pad(C, ldc, ldpc, -3.0)
    dA, dB, dC = (torch.from_numpy(x).cuda() for x in (bA, bB, bC))
    f = getattr(P.lib(), {2: "bnc_gemm_dd", 3: "bnc_gemm_td"}[K])
    vp = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    say("gemm padded K", K)
    assert f(m, n, k, vp(dA), lda, ldpa, vp(dB), ldb, ldpb, vp(dC), ldc, ldpc, None) == 0
    got = host(dC)
    exp = pad(want, ldc, ldpc, -3.0)
    np.testing.assert_array_equal(got, exp)
