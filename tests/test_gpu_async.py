"""bnc_refine_async, the refinement loop driven on the device: every
outcome (x, corrections, status, info, norms) equals bnc_refine's, bit for
bit, over the loop's exits (converged by either test, stagnated, out of
corrections, singular, non-finite input, a timed-out wait), both long
precisions and the split form; and the whole solve captured into a HIP
graph gives the same results on every replay, also after the right-hand
side has changed in place between replays."""
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


def run_async(P, A, b, K, **kw):
    import torch
    n = A.shape[1]
    lw = kw.get("long_words", 4)
    x = torch.full((lw, n), 7.0, dtype=torch.float64, device="cuda")
    work = torch.empty(P.refine_workspace_size(n, K), dtype=torch.uint8, device="cuda")
    res = torch.zeros(P.refine_result_bytes(), dtype=torch.uint8, device="cuda")
    P.refine_async(A, b, K, res, x, work, **kw)
    return x, P.refine_result(res)


def same(P, out, x, r):
    assert r["status"] == out["status"], (r["status"], out["status"])
    assert r["iters"] == out["iters"] and r["info"] == out["info"]
    np.testing.assert_array_equal(host(x), host(out["x"]))
    for f in ("resid_norm", "x_norm", "a_norm"):
        assert r[f] == out[f], (f, r[f], out[f])
    assert r["residual_inexact"] == out["residual_inexact"]


CASES = [
    ("randsvd", 300, 1e10, 2, {}),
    ("uniform", 200, 1.0, 3, {}),
    ("randsvd", 257, 1e10, 2, dict(ozaki=5)),
    ("randsvd", 130, 1e17, 1, dict(stagnation_ratio=0.5)),     # a binary64 factor stagnates
    ("randsvd", 96, 1e12, 2, dict(rtol=2.0 ** -209, ctol=0.0)),  # eq. (2) alone
    ("uniform", 64, 1.0, 4, dict(max_iter=0)),
    ("uniform", 65, 1.0, 2, dict(max_iter=1, ctol=0.0)),
]


@pytest.mark.parametrize("kind,n,cond,K,kw", CASES)
def test_async_equals_sync(P, kind, n, cond, K, kw):
    Ap, b, _ = synth.problem(kind, n, config=9, instance=n, cond=cond)
    dA, db = dev(Ap), dev(b)
    say("async vs sync", kind, n, cond, K, kw)
    out = P.refine(dA, db, K, **kw)
    x, r = run_async(P, dA, db, K, **kw)
    same(P, out, x, r)


def test_async_long_precision_paper_system(P):
    n = 100
    Ap, b, _, _ = synth.paper_problem(n)
    b8 = O.extend(b, 8)
    kw = dict(long_words=8, rtol=1e-100, ctol=0.0, max_iter=40)
    say("async 424-bit paper system")
    out = P.refine(dev(Ap), dev(b8), 3, **kw)
    x, r = run_async(P, dev(Ap), dev(b8), 3, **kw)
    same(P, out, x, r)
    assert r["status"] == P.BNC_CONVERGED


def test_async_failures(P):
    # exactly singular in every precision: two equal rows
    Ap, b, _ = synth.problem("uniform", 40, config=9, instance=1)
    Ap[0, :, 3] = Ap[0, :, 7]
    say("async singular")
    out = P.refine(dev(Ap), dev(b), 2)
    x, r = run_async(P, dev(Ap), dev(b), 2)
    same(P, out, x, r)
    assert r["status"] == P.BNC_SINGULAR and np.all(host(x) == 0.0)
    Ap2 = Ap.copy()
    Ap2[0, 5, 5] = np.nan
    say("async nonfinite")
    out = P.refine(dev(Ap2), dev(b), 2)
    x, r = run_async(P, dev(Ap2), dev(b), 2)
    same(P, out, x, r)
    assert r["status"] == P.BNC_NONFINITE


def test_async_timeout(P):
    Ap, b, _ = synth.problem("uniform", 128, config=9, instance=2)
    say("async forced timeout")
    P.test_force_timeout(2)
    try:
        x, r = run_async(P, dev(Ap), dev(b), 2)
    finally:
        P.test_force_timeout(0)
    assert r["status"] == P.BNC_TIMED_OUT


def test_async_graph_replays(P):
    import torch
    n, K = 128, 3
    Ap, b, _ = synth.problem("uniform", n, config=9, instance=3)
    Ap2, b2, _ = synth.problem("uniform", n, config=9, instance=4)
    dA, db = dev(Ap), dev(b)
    x = torch.zeros((4, n), dtype=torch.float64, device="cuda")
    work = torch.empty(P.refine_workspace_size(n, K), dtype=torch.uint8, device="cuda")
    res = torch.zeros(P.refine_result_bytes(), dtype=torch.uint8, device="cuda")
    P.refine_async(dA, db, K, res, x, work)  # outside the capture first (creates the side stream)
    torch.cuda.synchronize()
    ref1 = P.refine(dA, db, K)
    ref2 = P.refine(dA, dev(b2 * 0 + b2), K)  # a second right-hand side, same matrix
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    say("capture")
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s, capture_error_mode="thread_local"):
            P.refine_async(dA, db, K, res, x, work)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        say("replay", rep)
        x.fill_(3.0)
        res.zero_()
        want = ref1 if rep != 1 else ref2
        db.copy_(dev(b) if rep != 1 else dev(b2))
        g.replay()
        torch.cuda.synchronize()
        r = P.refine_result(res)
        same(P, want, x, r)
        # eager work between replays
        other = P.refine(dev(Ap2), dev(b2), 2)
        assert other["status"] == P.BNC_CONVERGED
