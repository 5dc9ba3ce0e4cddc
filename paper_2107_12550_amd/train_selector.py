"""Train the factor-precision selector on systems the method labels itself
and evaluate it against escalate-on-stagnation on a held-out stream.

  python -m paper_2107_12550_amd.train_selector --train 200000 --test 16384 \\
      --out model.npz --report report.json

The labelled training set can also be made in shards (each a separate
run: --shard-out shard.npz --first F --train C labels systems F..F+C-1 of
the training stream) and trained from them (--shards a.npz b.npz ...).

Training systems: seeded randsvd, n ~ U{32..512}, cond = 10^U(1, 60),
binary64 entries up to cond 1e15 and quad-double-word entries above (a
binary64 copy cannot hold a larger condition), b = A * ones exact (seed
stream 5); held-out systems the same law from seed stream 6.  Runs on one
GPU; prints progress per chunk.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=200000)
    ap.add_argument("--test", type=int, default=16384)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--chunk", type=int, default=4096)
    ap.add_argument("--n-lo", type=int, default=32)
    ap.add_argument("--n-hi", type=int, default=512)
    ap.add_argument("--words-above", type=float, default=1e15,
                    help="conditions above this keep quad-double-word entries (0: all binary64)")
    ap.add_argument("--out")
    ap.add_argument("--report")
    ap.add_argument("--first", type=int, default=0, help="first training system (with --shard-out)")
    ap.add_argument("--shard-out", help="label --train systems from --first, save them here and stop")
    ap.add_argument("--shards", nargs="*", help="train on these labelled shards instead of labelling now")
    args = ap.parse_args()
    if not args.shard_out and not (args.out and args.report):
        ap.error("--out and --report are required unless --shard-out is given")
    import torch

    from . import selector as SEL
    workers = min(16, os.cpu_count() or 1)
    t0 = time.perf_counter()
    if args.shards:
        parts = [np.load(p, allow_pickle=False) for p in args.shards]
        F = np.concatenate([z["F"] for z in parts])
        cls = np.concatenate([z["cls"] for z in parts])
        steps = np.concatenate([z["steps"] for z in parts])
        t_data = float(sum(float(z["seconds"]) for z in parts))
        args.train = int(sum(int(z["count"]) for z in parts))
    else:
        F, cls, steps = SEL.dataset(args.train, config=5, n_lo=args.n_lo, n_hi=args.n_hi, chunk=args.chunk,
                                    workers=workers, log=log, words_above=args.words_above or None,
                                    first=args.first)
        t_data = time.perf_counter() - t0
        if args.shard_out:
            np.savez(args.shard_out, F=F, cls=cls, steps=steps, seconds=t_data, count=args.train, first=args.first)
            log(f"[selector] shard of {args.train} systems from {args.first} saved to {args.shard_out}")
            return
    log(f"[selector] training set: {F.shape[0]} systems, classes {np.bincount(cls, minlength=4).tolist()}")
    Ft = torch.tensor(F, device="cuda")
    net, hist = SEL.train(Ft, torch.tensor(cls), torch.tensor(steps), epochs=args.epochs, log=log)
    SEL.save(net, args.out, meta=dict(train=int(F.shape[0]), epochs=args.epochs))
    pred, pst = SEL.predict(net, Ft)
    train_acc = float(np.mean(pred == cls))
    # held-out stream, evaluated chunk by chunk
    import synth
    tot = None
    labels = []
    for c0 in range(0, args.test, args.chunk):
        m = min(args.chunk, args.test - c0)
        As, bs, exact, _ = synth.batch(m, args.n_lo, args.n_hi, 1.0, 60.0, config=6, workers=workers, first=c0,
                                       words_above=args.words_above or None)
        dA = [torch.from_numpy(a).cuda() for a in As]
        db = [torch.from_numpy(b).cuda() for b in bs]
        r = SEL.evaluate(net, dA, db)
        lab = SEL.label(dA, db)
        Fh = SEL.bnc.features(dA, db)
        ph, _ = SEL.predict(net, Fh)
        labels.append((lab["cls"], ph))
        if tot is None:
            tot = {k: (v if not isinstance(v, list) else list(v)) for k, v in r.items()}
        else:
            for k, v in r.items():
                if isinstance(v, list):
                    tot[k] = [a + b for a, b in zip(tot[k], v)]
                elif k not in ("speedup", "speedup_vs_dd", "fallback_fraction"):
                    tot[k] += v
        log(f"[selector] held-out {c0 + m}/{args.test}: baseline {r['baseline_ms']:.1f} ms, "
            f"selector {r['selector_ms']:.1f} ms")
    lc = np.concatenate([a for a, _ in labels])
    lp = np.concatenate([b for _, b in labels])
    tot["speedup"] = tot["baseline_ms"] / tot["selector_ms"]
    tot["speedup_vs_dd"] = tot["dd_ms"] / tot["selector_ms"]
    tot["fallback_fraction"] = tot["selector_escalations"] / tot["count"]
    tot["under_predicted_fraction"] = float(np.mean(lp < lc))
    tot["heldout_accuracy"] = float(np.mean(lp == lc))
    tot["heldout_label_counts"] = np.bincount(lc, minlength=4).tolist()
    report = dict(workload=dict(n_lo=args.n_lo, n_hi=args.n_hi, cond="10^U(1, 60)",
                                quad_double_words_above=args.words_above or None, train=args.train, test=args.test),
                  train_systems=int(F.shape[0]), train_class_counts=np.bincount(cls, minlength=4).tolist(),
                  train_accuracy=train_acc, loss_history=hist, data_seconds=t_data, heldout=tot)
    with open(args.report, "w") as f:
        json.dump(report, f, indent=1)
    log(json.dumps(report["heldout"]))


if __name__ == "__main__":
    main()
