"""Writes the oracle's results for the batched workload (512 independent 1D
tempered problems, N log-uniform in [2^10, 2^15], 100 CN steps of
dt = 1e-3, PCG64 seed 8324) into this folder: every problem with
N <= 4096, and 32 of the larger ones drawn with PCG64 seed 358.

Calls only ``oracle/`` (the memory-lean dense CN of ``cn_run_lean``) and the
seeded input recipes of ``workloads``.  Each problem keeps u at the last step
on 512 positions drawn with PCG64(10000 + index) (all positions when N is
smaller) and the 2-norm of the whole vector, so that the GPU test can state
the error on the sample relative to the full norm.

    python tests/golden/make_batched_goldens.py            # both parts
    python tests/golden/make_batched_goldens.py small      # N <= 4096 only
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W                                   # noqa: E402
from oracle.levy_oracle import Problem, cn_run_lean     # noqa: E402

NAME = "batched512_sample"
NSMALL = 4096
NLARGE = 32
KEEP = 512


def oracle_problem(w):
    return Problem(dim=w.dim, n=w.n, lo=w.lo, hi=w.hi, a=w.a, b=tuple(w.b), c=w.c, s=w.s,
                   lam=w.lam, C=w.C, r0=w.r0)


def selection(ws):
    small = [i for i, w in enumerate(ws) if w.n <= NSMALL]
    large = [i for i, w in enumerate(ws) if w.n > NSMALL]
    rng = np.random.Generator(np.random.PCG64(358))
    picked = sorted(int(i) for i in rng.choice(large, NLARGE, replace=False))
    return small, picked


def positions(i, n):
    if n <= KEEP:
        return np.arange(n, dtype=np.int32)
    rng = np.random.Generator(np.random.PCG64(10000 + i))
    return np.sort(rng.choice(n, KEEP, replace=False)).astype(np.int32)


def main(parts):
    ws = W.config4_instances()
    small, large = selection(ws)
    todo = (small if "small" in parts else []) + (large if "large" in parts else [])
    path_npz = os.path.join(HERE, NAME + ".npz")
    path_json = os.path.join(HERE, NAME + ".json")
    out = dict(np.load(path_npz)) if os.path.exists(path_npz) else {}
    meta = json.load(open(path_json)) if os.path.exists(path_json) else {
        "name": NAME, "problems": len(ws), "small": small, "large": large, "keep": KEEP, "entries": {}}
    t0 = time.perf_counter()
    for k, i in enumerate(todo):
        if str(i) in meta["entries"]:
            continue
        w = ws[i]
        res = cn_run_lean(oracle_problem(w), w.dt, w.steps, w.u0)
        pos = positions(i, w.n)
        out["p%d" % i] = pos
        out["u%d" % i] = res.u[pos]
        meta["entries"][str(i)] = {"N": w.n, "steps": w.steps, "key": W.workload_key(w),
                                   "norm": float(np.linalg.norm(res.u)), "seconds": res.timings}
        print(f"problem {i}: N {w.n} ({k + 1}/{len(todo)}, {time.perf_counter() - t0:.0f}s)", flush=True)
        if (k + 1) % 16 == 0 or k + 1 == len(todo):
            np.savez_compressed(path_npz, **out)
            with open(path_json, "w") as f:
                json.dump(meta, f, indent=1)
    np.savez_compressed(path_npz, **out)
    with open(path_json, "w") as f:
        json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or ["small", "large"])
