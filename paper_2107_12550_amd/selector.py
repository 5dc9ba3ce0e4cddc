"""Learned choice of the factor precision (a project addition on top of the
paper's mixed-precision refinement, Kouya 2021 Sec. 2 / Listing 1).

The method labels its own training data: every system is refined with a
1-, 2-, 3- and 4-word factor (bnc_refine_batched, escalation off, stagnation
test on), and its class is the cheapest factor precision, by the device's
per-system time (minimum of two runs, costs within 5 % tie to fewer words),
whose refinement reaches the target accuracy (forward error against the
exact solution); its step count is the number of corrections that took.  A 24-64-64-5 network (bnc_mlp_*) learns class and
log2(1 + steps) from the 24 features of bnc_features.

In use, each system starts at the predicted precision; systems whose
refinement loop does not report convergence (stagnation or no convergence
within the correction limit: the loop's own status, the exact solution being
unknown in use) escalate one word at a time, which is the plain
escalate-on-stagnation rule started one or more rungs higher.  evaluate()
compares that with the rule started at one word and with a fixed start at
two words; afterwards, each path's solutions are checked against the exact
solution, and a system that converged to a wrong answer counts as a failure
of that path.

Every number is computed by the library's kernels; this module batches
systems, keeps the books and moves tensors.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from . import bnc

TARGET = 1e-45           # forward error the refinement must reach
CTOL = 2.0 ** -150       # forward test of the loop (about 7e-46)
STAG_RATIO = 0.5         # stagnation test of the loop
MAX_ITER = 30


def _events():
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def max_err_vs_ones(xs) -> np.ndarray:
    """max_i |x_i - 1| of each solution (exact solution all ones), from the
    quad-double words; device arithmetic in binary64."""
    dev = xs[0].device
    X = torch.cat([x.reshape(4, -1) for x in xs], dim=1)
    seg = torch.repeat_interleave(torch.arange(len(xs), device=dev),
                                  torch.tensor([x.shape[-1] for x in xs], device=dev))
    e = torch.abs(((X[0] - 1.0) + X[1]) + (X[2] + X[3]))
    out = torch.zeros(len(xs), dtype=torch.float64, device=dev)
    out.scatter_reduce_(0, seg, e, reduce="amax", include_self=True)
    return out.cpu().numpy()


def solve_at(As, bs, K: int) -> dict:
    """Refine every system with a K-word factor: one batched launch for the
    orders up to 256 (256 threads per workgroup) and one for those above
    (512), back to back."""
    count = len(As)
    ns = np.array([int(a.shape[-1]) for a in As])
    groups = [g for g in (np.nonzero(ns <= 256)[0], np.nonzero(ns > 256)[0]) if g.size]
    solvers = [(g, bnc.BatchSolver([As[i] for i in g], [bs[i] for i in g], K, max_iter=MAX_ITER, ctol=CTOL,
                                   stagnation_ratio=STAG_RATIO, threads=256 if ns[g].max() <= 256 else 512))
               for g in groups]
    e0, e1 = _events()
    e0.record()
    for _, S in solvers:
        S.run()
    e1.record()
    status = np.zeros(count, dtype=np.int32)
    iters = np.zeros(count, dtype=np.int64)
    lat = np.zeros(count)
    err = np.zeros(count)
    xs = [None] * count
    khz = bnc.wall_clock_khz()
    for g, S in solvers:
        res = S.results()
        status[g] = res["status"]
        iters[g] = res["iters"]
        lat[g] = (res["t_end"].astype(np.float64) - res["t_start"].astype(np.float64)) / khz
        err[g] = max_err_vs_ones(S.xs)
        for j, i in enumerate(g):
            xs[i] = S.xs[j]
        S.close()
    ms = e0.elapsed_time(e1)
    converged = status == bnc.BNC_CONVERGED
    ok = converged & (err <= TARGET)
    return dict(ok=ok, converged=converged, iters=iters, status=status, latency_ms=lat, total_ms=ms, xs=xs, err=err)


TIE = 1.05              # costs within 5 % count as a tie (fewer words win)


def label(As, bs, repeats: int = 2) -> dict:
    """Class (0..3 = 1..4 words) and step count of each system: the fewest
    words whose refinement reaches TARGET at a per-system device time within
    TIE of the cheapest successful precision (each time the minimum over
    `repeats` runs, which are bit-identical); systems no precision solves
    get class 3 and MAX_ITER steps."""
    count = len(As)
    cost = np.full((4, count), np.inf)
    iters = np.zeros((4, count), dtype=np.int64)
    per_k = {}
    for K in (1, 2, 3, 4):
        lat = None
        for _ in range(repeats):
            r = solve_at(As, bs, K)
            lat = r["latency_ms"] if lat is None else np.minimum(lat, r["latency_ms"])
        per_k[K] = dict(ok=r["ok"], latency_ms=lat, iters=r["iters"], total_ms=r["total_ms"])
        cost[K - 1] = np.where(r["ok"], lat, np.inf)
        iters[K - 1] = r["iters"]
    best = cost.min(axis=0)
    solved = np.isfinite(best)
    within = cost <= TIE * best[None, :]
    cls = np.where(solved, np.argmax(within, axis=0), 3).astype(np.int32)
    steps = np.where(solved, iters[cls, np.arange(count)], MAX_ITER)
    return dict(cls=cls, steps=steps, per_k=per_k, solved=solved)


def step_target(steps) -> np.ndarray:
    return np.log2(1.0 + np.asarray(steps, dtype=np.float64))


def init_params(seed: int) -> np.ndarray:
    """He-normal weights, zero biases, in the packed layout of bnc_mlp_*."""
    g = np.random.default_rng(seed)
    parts = []
    for fan_in, fan_out in ((24, 64), (64, 64), (64, 5)):
        parts.append(g.normal(0.0, math.sqrt(2.0 / fan_in), fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def train(F: torch.Tensor, cls: torch.Tensor, steps: torch.Tensor, epochs: int = 40, batch: int = 1024,
          lr: float = 2e-3, seed: int = 0, log=None) -> tuple[bnc.MLP, list]:
    """Adam on mini-batches; the input normalisation is the training set's
    per-feature mean and 1/std (std floored at 1e-3)."""
    dev = F.device
    mean = F.mean(dim=0)
    std = F.std(dim=0).clamp_min(1e-3)
    norm = torch.cat([mean, 1.0 / std]).to(torch.float32)
    net = bnc.MLP(torch.tensor(init_params(seed), device=dev), norm)
    tgt = torch.tensor(step_target(steps.cpu().numpy()), dtype=torch.float32, device=dev)
    cls = cls.to(torch.int32).to(dev)
    g = np.random.default_rng(seed + 1)
    N = F.shape[0]
    history = []
    for ep in range(epochs):
        perm = torch.tensor(g.permutation(N), device=dev)
        tot = torch.zeros(1, dtype=torch.float32, device=dev)
        nb = 0
        for s in range(0, N - batch + 1 if N >= batch else 1, batch):
            idx = perm[s:s + batch]
            tot += net.grad(F[idx], cls[idx], tgt[idx])
            net.adam(lr=lr)
            nb += 1
        history.append(float(tot.item()) / max(nb, 1))
        if log:
            log(f"[selector] epoch {ep + 1}/{epochs} loss {history[-1]:.4f}")
    return net, history


def predict(net: bnc.MLP, F: torch.Tensor):
    """(class 0..3, predicted corrections) per system."""
    out = net.forward(F)
    cls = torch.argmax(out[:, :4], dim=1).cpu().numpy().astype(np.int32)
    st = np.maximum(np.exp2(out[:, 4].cpu().numpy().astype(np.float64)) - 1.0, 0.0)
    return cls, st


def escalate_from(As, bs, start_words) -> dict:
    """Refine each system starting at its start precision; those whose loop
    does not report convergence (its own status: stagnated or out of
    corrections) move up one word and are refined again (one batched launch
    per precision, in increasing order).  The exact solution plays no part
    in the decisions; afterwards each returned solution is checked against
    it.  Returns total device time, per-system final precision, number of
    escalations, `solved` (the loop converged) and `accurate` (converged
    and within TARGET of the exact solution)."""
    count = len(As)
    cur = np.asarray(start_words, dtype=np.int64).copy()
    done = np.zeros(count, dtype=bool)
    conv_all = np.zeros(count, dtype=bool)
    acc_all = np.zeros(count, dtype=bool)
    total = 0.0
    launches = 0
    escal = 0
    for K in (1, 2, 3, 4):
        idx = np.nonzero((cur == K) & ~done)[0]
        if idx.size == 0:
            continue
        r = solve_at([As[i] for i in idx], [bs[i] for i in idx], K)
        total += r["total_ms"]
        launches += 1
        good = r["converged"]
        done[idx[good]] = True
        conv_all[idx[good]] = True
        acc_all[idx[good]] = r["err"][good] <= TARGET
        bad = idx[~good]
        if K < 4:
            cur[bad] = K + 1
            escal += bad.size
        else:
            done[bad] = True
    return dict(total_ms=total, launches=launches, escalations=int(escal), final_words=cur, solved=conv_all,
                accurate=acc_all)


def evaluate(net: bnc.MLP, As, bs) -> dict:
    """Selector (features + inference + escalation from the predicted
    precision) against the escalate-on-stagnation rule from one word and
    from a fixed two words (double-double).  `*_solved`: systems whose loop
    converged; `*_wrong`: of those, the ones whose solution misses TARGET
    against the exact solution (failures of that path)."""
    base = escalate_from(As, bs, np.ones(len(As), dtype=np.int64))
    dd = escalate_from(As, bs, np.full(len(As), 2, dtype=np.int64))
    e0, e1 = _events()
    e0.record()
    F = bnc.features(As, bs)
    cls, st = predict(net, F)
    e1.record()
    torch.cuda.synchronize()
    t_pred = e0.elapsed_time(e1)
    sel = escalate_from(As, bs, cls.astype(np.int64) + 1)
    return dict(
        count=len(As),
        baseline_ms=base["total_ms"], baseline_escalations=base["escalations"],
        baseline_solved=int(base["solved"].sum()),
        baseline_wrong=int((base["solved"] & ~base["accurate"]).sum()),
        dd_ms=dd["total_ms"], dd_escalations=dd["escalations"], dd_solved=int(dd["solved"].sum()),
        dd_wrong=int((dd["solved"] & ~dd["accurate"]).sum()), dd_attempts=int(len(As) + dd["escalations"]),
        selector_ms=t_pred + sel["total_ms"], selector_predict_ms=t_pred, selector_solve_ms=sel["total_ms"],
        selector_escalations=sel["escalations"], selector_solved=int(sel["solved"].sum()),
        selector_wrong=int((sel["solved"] & ~sel["accurate"]).sum()),
        fallback_fraction=float(np.mean(sel["final_words"] != cls + 1)),
        baseline_attempts=int(len(As) + base["escalations"]), selector_attempts=int(len(As) + sel["escalations"]),
        predicted_class_counts=np.bincount(cls, minlength=4).tolist(),
        baseline_final_counts=np.bincount(base["final_words"] - 1, minlength=4).tolist(),
        speedup=base["total_ms"] / max(t_pred + sel["total_ms"], 1e-9),
        speedup_vs_dd=dd["total_ms"] / max(t_pred + sel["total_ms"], 1e-9),
    )


def save(net: bnc.MLP, path: str, meta: dict | None = None):
    np.savez(path, params=net.params.cpu().numpy(), norm=net.norm.cpu().numpy(),
             meta=np.array(repr(meta or {})))


def load(path: str, device="cuda") -> bnc.MLP:
    z = np.load(path, allow_pickle=False)
    return bnc.MLP(torch.tensor(z["params"], device=device), torch.tensor(z["norm"], device=device))


def dataset(count: int, config: int, n_lo: int = 32, n_hi: int = 512, lc_lo: float = 1.0, lc_hi: float = 60.0,
            chunk: int = 4096, workers: int = 16, log=None, words_above: float | None = 1e15, first: int = 0):
    """Generate, label and featurise `count` seeded randsvd systems in chunks
    (binary64 entries up to cond `words_above`, quad-double words above;
    exact right-hand side A * ones), systems first .. first + count - 1 of
    the seed stream.  Returns host arrays F (count, 24), cls and steps."""
    import synth
    Fs, cs, ss = [], [], []
    t0 = time.perf_counter()
    for c0 in range(0, count, chunk):
        m = min(chunk, count - c0)
        As, bs, exact, _ = synth.batch(m, n_lo, n_hi, lc_lo, lc_hi, config=config, workers=workers,
                                       first=first + c0, words_above=words_above)
        dA = [torch.from_numpy(a).cuda() for a in As]
        db = [torch.from_numpy(b).cuda() for b in bs]
        lab = label(dA, db)
        F = bnc.features(dA, db).cpu().numpy()
        keep = np.asarray(exact, dtype=bool)
        Fs.append(F[keep])
        cs.append(lab["cls"][keep])
        ss.append(lab["steps"][keep])
        del dA, db
        if log:
            log(f"[selector] {c0 + m}/{count} systems labelled, {time.perf_counter() - t0:.1f} s, "
                f"classes so far {np.bincount(np.concatenate(cs), minlength=4).tolist()}")
    return np.concatenate(Fs), np.concatenate(cs), np.concatenate(ss)
