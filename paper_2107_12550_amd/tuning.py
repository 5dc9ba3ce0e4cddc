"""Autotuning of the batched refined solves (bnc_refine_batched).

The batched kernel has two launch-shape knobs that leave every result
unchanged: the LU panel width (4, 8 or 16 columns staged in LDS) and the number
of threads per workgroup (64, 128, 256 or 512; one thread per row, so a
workgroup takes systems up to that order, and smaller workgroups let more
small systems run at once).  tune() times every variant that fits each size
class on a seeded sample of that class and keeps the fastest; the plan is a
small JSON-able dict.  TunedBatchSolver splits a batch by size class and
runs one launch per class with its variant, all captured in one graph.
"""
from __future__ import annotations

import json

import numpy as np
import torch

from . import bnc

CLASSES = ((1, 64), (65, 128), (129, 256), (257, 512))
PANELS = (4, 8, 16)
THREADS = (64, 128, 256, 512)


def _time(fn, reps: int) -> float:
    best = float("inf")
    for _ in range(reps):
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def tune(K: int, sample: int = 1024, reps: int = 3, ctol: float = 2.0 ** -150, config: int = 9,
         lc_lo: float = 2.0, lc_hi: float = 30.0, log=None, words_above: float | None = 1e15,
         classes=CLASSES) -> dict:
    """Time every (panel, threads) variant on `sample` seeded randsvd systems
    per size class (cond = 10^U(lc_lo, lc_hi), quad-double-word entries
    above `words_above`), then check whether the classes up to 256 run
    faster as one launch with the largest of them's variant (no drain
    between launches) than one launch each, and merge them if so; returns
    the plan."""
    import synth
    out = []
    pool = []  # the sampled systems of the classes up to 256
    for ci, (lo, hi) in enumerate(classes):
        As, bs, _, _ = synth.batch(sample, max(lo, 2), hi, lc_lo, lc_hi, config=config, workers=16,
                                   first=ci * sample, words_above=words_above)
        dA = [torch.from_numpy(a).cuda() for a in As]
        db = [torch.from_numpy(b).cuda() for b in bs]
        if hi <= 256:
            pool.append((dA, db))
        trials = []
        for nt in THREADS:
            if nt < hi:
                continue
            for pw in PANELS:
                S = bnc.BatchSolver(dA, db, K, ctol=ctol, panel=pw, threads=nt)
                ms = _time(S.run, reps)
                trials.append(dict(panel=pw, threads=nt, slots=S.slots, ms=ms))
                if log:
                    log(f"[tune] K={K} n in [{lo},{hi}] panel {pw} threads {nt} slots {S.slots}: {ms:.3f} ms")
        best = min(trials, key=lambda d: d["ms"])
        out.append(dict(n_lo=lo, n_hi=hi, panel=best["panel"], threads=best["threads"], trials=trials))
    plan = dict(K=K, sample=sample, classes=out)
    small = [c for c in out if c["n_hi"] <= 256]
    if len(small) > 1:
        dA = [a for p in pool for a in p[0]]
        db = [b for p in pool for b in p[1]]
        big = max(small, key=lambda c: c["n_hi"])
        split = TunedBatchSolver(dA, db, K, dict(K=K, classes=small), ctol=ctol)
        ms_split = _time(lambda: split.run(graph=True), reps)
        one = bnc.BatchSolver(dA, db, K, ctol=ctol, panel=big["panel"], threads=big["threads"])
        ms_one = _time(lambda: one.run(graph=True), reps)
        if log:
            log(f"[tune] orders up to 256: one launch per class {ms_split:.3f} ms, one launch "
                f"(panel {big['panel']}, threads {big['threads']}) {ms_one:.3f} ms")
        plan["merge"] = dict(split_ms=ms_split, one_ms=ms_one)
        if ms_one < ms_split:
            rest = [c for c in out if c["n_hi"] > 256]
            plan["classes"] = [dict(n_lo=small[0]["n_lo"], n_hi=big["n_hi"], panel=big["panel"],
                                    threads=big["threads"], trials=[])] + rest
    return plan


def save_plan(plan: dict, path: str):
    with open(path, "w") as f:
        json.dump(plan, f, indent=1)


def load_plan(path: str) -> dict:
    with open(path) as f:
        return json.load(f)


class TunedBatchSolver:
    """Batched refined solves split by size class, each class launched with
    its tuned variant; run(graph=True) replays one captured graph holding
    every class's launch."""

    def __init__(self, As, bs, K: int, plan: dict, **kw):
        if plan.get("K") != K:
            raise bnc.BncError("TunedBatchSolver: plan was tuned for another factor precision")
        ns = np.array([int(a.shape[-1]) for a in As])
        self.count = len(As)
        self.parts = []
        for c in plan["classes"]:
            idx = np.nonzero((ns >= c["n_lo"]) & (ns <= c["n_hi"]))[0]
            if idx.size:
                S = bnc.BatchSolver([As[i] for i in idx], [bs[i] for i in idx], K, panel=c["panel"],
                                    threads=c["threads"], **kw)
                self.parts.append((idx, S))
        covered = sum(i.size for i, _ in self.parts)
        if covered != self.count:
            raise bnc.BncError("TunedBatchSolver: some orders are outside the plan's classes")
        self.xs = [None] * self.count
        for idx, S in self.parts:
            for j, i in enumerate(idx):
                self.xs[i] = S.xs[j]
        self.graph = None

    def run(self, graph: bool = False):
        if not graph:
            for _, S in self.parts:
                S.run()
            return
        if self.graph is None:
            self.stream = torch.cuda.Stream()
            self.graph = torch.cuda.CUDAGraph()
            self.stream.wait_stream(torch.cuda.current_stream())
            with torch.cuda.graph(self.graph, stream=self.stream, capture_error_mode="relaxed"):
                for _, S in self.parts:
                    S.run()
            torch.cuda.current_stream().wait_stream(self.stream)
        self.graph.replay()

    def results(self):
        out = None
        for idx, S in self.parts:
            r = S.results()
            if out is None:
                out = np.zeros(self.count, dtype=r.dtype)
            out[idx] = r
        return out

    @property
    def slots(self):
        return [S.slots for _, S in self.parts]
