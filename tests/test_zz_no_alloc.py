"""The no-allocation solve bnc_getrs_noalloc (fixed device scratch inside
the library) against the workspace entry point bnc_getrs_*, bit for bit,
through the C-ABI: two calls in a row, the second on a smaller system (so
the shared scratch holds the first call's contents), several right-hand
sides, and the size limit."""
import ctypes
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_12550_amd as P
    L = P.lib()
    L.bnc_getrs_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.c_void_p]
    L.bnc_getrs_noalloc.restype = ctypes.c_int
    return P


SUFFIX = {1: "d", 2: "dd", 3: "td", 4: "qd"}


def solve_both(P, K, n, nrhs, seed):
    import torch
    vp = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    L = P.lib()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    Ap, b, _ = synth.problem("uniform", n, config=0, instance=seed)
    A = torch.zeros((K, n, n), dtype=torch.float64, device="cuda")
    A[:1].copy_(torch.from_numpy(Ap))
    ipiv, info = P.getrf(K, A)
    assert int(info.item()) == 0
    g = np.random.default_rng(seed)
    B0 = torch.from_numpy(g.uniform(-1, 1, (K, nrhs, n))).cuda()
    B0[1:] *= 2.0 ** -60
    # the workspace entry point
    Bw = B0.clone()
    infw = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    work = torch.empty(P.getrs_workspace_size(K, n), dtype=torch.uint8, device="cuda")
    f = getattr(L, f"bnc_getrs_{SUFFIX[K]}")
    assert f(n, nrhs, vp(A), n, n * n, vp(ipiv), vp(Bw), n, n * nrhs, vp(infw), vp(work), work.numel(), stream) == 0
    # the no-allocation entry point
    Bn = B0.clone()
    infn = torch.full((1,), 5, dtype=torch.int64, device="cuda")
    say("noalloc K", K, "n", n, "nrhs", nrhs)
    rc = L.bnc_getrs_noalloc(K, n, nrhs, vp(A), n, n * n, vp(ipiv), vp(Bn), n, n * nrhs, vp(infn), stream)
    assert rc == 0, L.bnc_last_error()
    torch.cuda.synchronize()
    assert int(infw.item()) == 0 and int(infn.item()) == 0
    np.testing.assert_array_equal(Bn.cpu().numpy(), Bw.cpu().numpy())
    assert np.isfinite(Bn.cpu().numpy()).all()


@pytest.mark.parametrize("K", [2, 3, 4, 1])
def test_noalloc_equals_workspace_entry_point_twice(P, K):
    solve_both(P, K, 300, 2, 500 + K)
    solve_both(P, K, 130, 1, 600 + K)  # smaller: the scratch holds the first call's words


def test_noalloc_size_limit(P):
    L = P.lib()
    rc = L.bnc_getrs_noalloc(2, 16385, 1, 1 << 20, 16385, 16385 * 16385, 2 << 20, 3 << 20, 16385, 16385, None, None)
    assert rc == P.BNC_ERR_UNSUPPORTED
    assert b"16384" in L.bnc_last_error()
    assert L.bnc_getrs_noalloc(5, 8, 1, None, 8, 64, None, None, 8, 8, None, None) == -1
    assert L.bnc_getrs_noalloc(2, -1, 1, None, 8, 64, None, None, 8, 8, None, None) == -2
