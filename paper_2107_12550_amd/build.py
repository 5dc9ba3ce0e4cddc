"""Build libbnc.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["getrf.hip", "ozaki.hip", "getrs.hip", "refine.hip", "batch.hip", "selector.hip", "api.hip"]
# (source, object, extra flags): the batched solver is compiled once per
# factor word count, so its four units compile in parallel with the rest
UNITS = [(s, s.replace(".hip", ".o"), []) for s in SOURCES if s != "batch.hip"] + [
    ("batch.hip", f"batch_k{k}.o", [f"-DBNC_BATCH_K={k}"]) for k in (1, 2, 3, 4)]
LIB = os.path.join(HERE, "libbnc.so")
ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # every rounding happens as written: no contraction into FMA
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    objs = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    procs = []
    for src, o, extra in UNITS:
        obj = os.path.join(bdir, o)
        cmd = ["hipcc", *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
    for p, src in procs:
        _, err = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(err)
            raise RuntimeError(f"hipcc failed on {src}")
        if verbose and err.strip():
            sys.stderr.write(err)
    tmp = LIB + ".tmp"
    subprocess.check_call(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
