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
