"""GPU parity of the batched refined solves (bnc_refine_batched) with the
oracle: every system of a mixed batch (binary64 and quad-double-word
entries, orders 1..512) must come out bit for bit as the oracle's
Listing-1 refinement of that system alone, whatever the order the systems
are taken in, also through a captured HIP graph."""
import sys

import numpy as np
import pytest

import oracle as O
import synth
from helpers import dev

pytestmark = pytest.mark.gpu

CTOL = 2.0 ** -150  # refine to ~1e-45 (the batched workload's target)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_2107_12550_amd as P
    return P


def mixed_batch():
    sizes = [1, 2, 5, 16, 33, 64, 65, 97, 128, 130, 200, 256]
    As, bs = [], []
    for i, n in enumerate(sizes):
        kind = "uniform" if i % 3 == 0 else "randsvd"
        cond = [1e3, 1e10, 1e15, 1e30][i % 4]
        Ap, b, _ = synth.problem(kind, n, config=3, instance=500 + i, cond=cond)
        As.append(Ap)
        bs.append(b)
    # an exactly singular system and one with a NaN
    A = np.array([[2.0, 1, 0, 1], [1, 3, 1, 0], [0, 1, 4, 1], [1, 3, 1, 0]])
    Ap = synth.planes(A)
    b, _ = synth.rhs_ones(Ap)
    As.append(Ap)
    bs.append(b)
    Ap2, b2, _ = synth.problem("uniform", 20, config=3, instance=599)
    Ap2 = Ap2.copy()
    Ap2[0, 3, 4] = np.nan
    As.append(Ap2)
    bs.append(b2)
    return As, bs


def words_batch():
    """Quad-double-word systems (conditions a binary64 copy cannot hold),
    binary64 ones beside them, and orders above 256."""
    specs = [(40, 1e20, True), (97, 1e25, True), (130, 1e30, True), (64, 1e8, False), (257, 1e25, True),
             (300, 1e12, False), (389, 1e28, True), (512, 1e5, False)]
    As, bs = [], []
    for i, (n, cond, words) in enumerate(specs):
        Ap, b, _ = synth.problem("randsvd_words" if words else "randsvd", n, config=3, instance=900 + i, cond=cond)
        As.append(Ap)
        bs.append(b)
    return As, bs


def check_vs_oracle(S, refs):
    res = S.results()
    for i, ref in enumerate(refs):
        assert res["status"][i] == ref["status"], i
        if ref["status"] == O.SINGULAR:
            assert res["info"][i] == ref["info"]
        assert res["iters"][i] == ref["iters"], i
        assert res["residual_inexact"][i] == 0
        np.testing.assert_array_equal(S.xs[i].cpu().numpy(), ref["x"], err_msg=f"system {i}")


@pytest.mark.parametrize("K", [2, 3])
def test_batched_words_and_large_orders_vs_oracle(P, K):
    """Quad-double-word A staged to K words, its exact residual over every
    word, and orders up to 512 (512 threads per workgroup)."""
    As, bs = words_batch()
    refs = [O.refine(A, b, K, ctol=CTOL) for A, b in zip(As, bs)]
    say("batched words/large K", K, "orders", [a.shape[-1] for a in As], "words", [a.shape[0] for a in As])
    S = P.BatchSolver([dev(A) for A in As], [dev(b) for b in bs], K, ctol=CTOL)
    assert S.opts.batch_threads == 512
    S.run()
    check_vs_oracle(S, refs)
    # the systems of order <= 256 again, in a 256-thread launch
    small = [i for i, a in enumerate(As) if a.shape[-1] <= 256]
    say("batched words K", K, "256 threads")
    S2 = P.BatchSolver([dev(As[i]) for i in small], [dev(bs[i]) for i in small], K, ctol=CTOL, threads=256)
    S2.run()
    check_vs_oracle(S2, [refs[i] for i in small])


def test_batched_four_words_512_threads_panel_fallback(P):
    """K = 4 at 512 threads: an 8-wide panel would not fit the LDS, the
    launch takes 4-wide panels, and the words are those of the oracle."""
    As, bs = words_batch()
    sel = [0, 4, 7]
    As, bs = [As[i] for i in sel], [bs[i] for i in sel]
    refs = [O.refine(A, b, 4, ctol=CTOL) for A, b in zip(As, bs)]
    for pw in (8, 4):
        say("batched K 4 threads 512 panel", pw)
        S = P.BatchSolver([dev(A) for A in As], [dev(b) for b in bs], 4, ctol=CTOL, panel=pw, threads=512)
        S.run()
        check_vs_oracle(S, refs)


def test_words_and_large_orders_through_a_graph(P):
    """The quad-double-word batch with orders up to 512 (512 threads per
    workgroup) through a captured HIP graph, replayed twice with the
    solutions overwritten in between: every replay equals the eager run
    word for word."""
    As, bs = words_batch()
    K = 3
    say("words batch eager")
    S = P.BatchSolver([dev(A) for A in As], [dev(b) for b in bs], K, ctol=CTOL)
    S.run()
    r0 = S.results()
    x0 = [x.cpu().numpy() for x in S.xs]
    for rep in range(2):
        for x in S.xs:
            x.fill_(5.0)
        say("words batch graph replay", rep)
        S.run(graph=True)
        r = S.results()
        assert np.array_equal(r["status"], r0["status"]) and np.array_equal(r["iters"], r0["iters"])
        for a, b in zip(x0, S.xs):
            np.testing.assert_array_equal(a, b.cpu().numpy())
    S.close()


@pytest.mark.parametrize("K", [2, 3])
def test_batched_bitexact_vs_oracle(P, K):
    As, bs = mixed_batch()
    refs = [O.refine(A, b, K, ctol=CTOL) for A, b in zip(As, bs)]
    say("batched K", K, "systems", len(As))
    S = P.BatchSolver([dev(A) for A in As], [dev(b) for b in bs], K, ctol=CTOL)
    S.run()
    res = S.results()
    for i, ref in enumerate(refs):
        assert res["status"][i] == ref["status"], i
        if ref["status"] == O.SINGULAR:
            assert res["info"][i] == ref["info"]
        assert res["iters"][i] == ref["iters"], i
        assert res["residual_inexact"][i] == 0
        np.testing.assert_array_equal(S.xs[i].cpu().numpy(), ref["x"], err_msg=f"system {i}")
        assert res["t_end"][i] >= res["t_start"][i]


def test_batched_order_independent_and_graph(P):
    As, bs = mixed_batch()
    K = 3
    say("batched identity order")
    S1 = P.BatchSolver([dev(A) for A in As], [dev(b) for b in bs], K, ctol=CTOL, order=list(range(len(As))))
    S1.run()
    r1 = S1.results()
    x1 = [x.cpu().numpy() for x in S1.xs]
    say("batched graph, reversed order, 2 replays")
    S2 = P.BatchSolver([dev(A) for A in As], [dev(b) for b in bs], K, ctol=CTOL,
                       order=list(reversed(range(len(As)))), slots=7)
    for rep in range(2):
        for x in S2.xs:
            x.fill_(123.0)
        S2.run(graph=True)
        r2 = S2.results()
        assert np.array_equal(r1["status"], r2["status"]) and np.array_equal(r1["iters"], r2["iters"])
        for a, b in zip(x1, S2.xs):
            np.testing.assert_array_equal(a, b.cpu().numpy())
    S2.close()


def test_batched_bad_size(P):
    """Orders above the launch's threads (and above 512) and word counts
    other than 1 or 4 are refused per system; the others still solve."""
    import torch
    K = 3
    A1, b1, _ = synth.problem("uniform", 300, config=3, instance=777)
    A2, b2, _ = synth.problem("uniform", 600, config=3, instance=778)
    A3, b3, _ = synth.problem("uniform", 30, config=3, instance=779)
    A4 = np.concatenate([A3, np.zeros_like(A3)])  # two words per entry
    say("batched bad size, 256 threads")
    S = P.BatchSolver([dev(A1), dev(A3)], [dev(b1), dev(b3)], K, ctol=CTOL, threads=256)
    S.run()
    assert list(S.results()["status"]) == [P.BNC_BAD_SIZE, P.BNC_CONVERGED]
    say("batched bad size, 512 threads")
    S = P.BatchSolver([dev(A2), dev(A1), dev(A4)], [dev(b2), dev(b1), dev(b3)], K, ctol=CTOL)
    S.run()
    assert list(S.results()["status"]) == [P.BNC_BAD_SIZE, P.BNC_CONVERGED, P.BNC_BAD_SIZE]
    torch.cuda.synchronize()


def test_launch_variants_bitexact(P):
    """Panel width and threads per workgroup are tuning knobs only: every
    variant returns the same words as the oracle-checked default, and a
    system above a variant's order limit is refused."""
    As, bs = mixed_batch()
    K = 2
    ns = [a.shape[-1] for a in As]
    ref = P.BatchSolver([dev(A) for A in As], [dev(b) for b in bs], K, ctol=CTOL)
    ref.run()
    r0 = ref.results()
    x0 = [x.cpu().numpy() for x in ref.xs]
    for nt in (64, 128, 256, 512):
        for pw in (4, 8, 16):
            say("variant threads", nt, "panel", pw)
            S = P.BatchSolver([dev(A) for A in As], [dev(b) for b in bs], K, ctol=CTOL, panel=pw, threads=nt)
            S.run()
            r = S.results()
            for i, n in enumerate(ns):
                if n > nt:
                    assert r["status"][i] == P.BNC_BAD_SIZE
                    continue
                assert r["status"][i] == r0["status"][i] and r["iters"][i] == r0["iters"][i], (nt, pw, i)
                np.testing.assert_array_equal(S.xs[i].cpu().numpy(), x0[i])


def test_tuned_solver_graph_replays(P):
    """A plan that sends each size class to its own variant, eager and
    through a captured graph replayed three times with eager work in
    between: every system equals the oracle's refine of it alone."""
    import torch
    from paper_2107_12550_amd import tuning
    As, bs = mixed_batch()
    K = 3
    refs = [O.refine(A, b, K, ctol=CTOL) for A, b in zip(As, bs)]
    plan = dict(K=K, classes=[dict(n_lo=1, n_hi=64, panel=4, threads=64),
                              dict(n_lo=65, n_hi=128, panel=8, threads=128),
                              dict(n_lo=129, n_hi=256, panel=4, threads=256)])
    T = tuning.TunedBatchSolver([dev(A) for A in As], [dev(b) for b in bs], K, plan, ctol=CTOL)
    say("tuned eager")
    T.run()
    for rep in range(4):
        res = T.results()
        for i, ref in enumerate(refs):
            assert res["status"][i] == ref["status"] and res["iters"][i] == ref["iters"], (rep, i)
            if ref["status"] != O.SINGULAR:
                np.testing.assert_array_equal(T.xs[i].cpu().numpy(), ref["x"], err_msg=f"rep {rep} system {i}")
        for x in T.xs:
            x.fill_(7.0)
        torch.cuda.synchronize()
        say("tuned graph replay", rep)
        T.run(graph=True)
        torch.cuda.synchronize()


def test_tune_smoke(P):
    from paper_2107_12550_amd import tuning
    say("tune smoke")
    plan = tuning.tune(2, sample=16, reps=1)
    # the classes tile 1..512 in order: the tuned ones, or those up to 256
    # merged into one launch when that was faster
    cl = [(c["n_lo"], c["n_hi"]) for c in plan["classes"]]
    assert cl == list(tuning.CLASSES) or cl == [(1, 256), (257, 512)], cl
    assert "merge" in plan and plan["merge"]["split_ms"] > 0 and plan["merge"]["one_ms"] > 0
    for c in plan["classes"]:
        assert c["threads"] >= c["n_hi"] and c["panel"] in tuning.PANELS
        assert c["trials"] or (c["n_lo"], c["n_hi"]) == (1, 256)
