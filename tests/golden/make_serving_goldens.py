"""Writes the oracle's results for the seeded 1 % sample of the serving
trace (200 requests/s for 60 s, PCG64 seeds 355 trace / 356 operator pool /
357 sample) into this folder.

Calls only ``oracle/`` (dense generator, CN by dense LU) and the seeded
input recipes of ``workloads``.  Requests whose N is at most NMAX get the
oracle's u at their last step; the others are listed with their sizes (the
GPU test compares them with the library's FP64 single-problem path).

    python tests/golden/make_serving_goldens.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W                                     # noqa: E402
from oracle.levy_oracle import Problem, cn_run, generator_dense   # noqa: E402

NMAX = 12000
NAME = "serve_poisson200_60s_sample"


def sample_indices(trace, seed=357, frac=0.01):
    rng = np.random.Generator(np.random.PCG64(seed))
    k = int(round(frac * len(trace)))
    return np.sort(rng.choice(len(trace), size=k, replace=False))


def main():
    tr = W.serving_trace()
    idx = sample_indices(tr)
    out, meta = {}, {"name": NAME, "trace_requests": len(tr), "sample": [int(i) for i in idx], "nmax": NMAX,
                     "oracle": {}, "gpu_only": {}}
    t0 = time.perf_counter()
    for i in idx:
        r = tr[int(i)]
        w = r["w"].with_(u0=W.request_u0(r))
        N = w.n if w.dim == 1 else w.n * w.n
        key = W.workload_key(w)
        if N > NMAX:
            meta["gpu_only"][str(int(i))] = {"N": N, "steps": r["steps"], "key": key}
            continue
        p = Problem(dim=w.dim, n=w.n, lo=w.lo, hi=w.hi, a=w.a, b=tuple(w.b), c=w.c, s=w.s, lam=w.lam, C=w.C,
                    r0=w.r0)
        u = cn_run(generator_dense(p), w.dt, r["steps"], w.u0).u
        out["r%d" % int(i)] = u
        meta["oracle"][str(int(i))] = {"N": N, "steps": r["steps"], "key": key}
        print(f"request {int(i)}: dim {w.dim} N {N} steps {r['steps']} ({time.perf_counter() - t0:.0f}s)",
              flush=True)
    np.savez_compressed(os.path.join(HERE, NAME + ".npz"), **out)
    meta["seconds"] = time.perf_counter() - t0
    with open(os.path.join(HERE, NAME + ".json"), "w") as f:
        json.dump(meta, f, indent=1)


if __name__ == "__main__":
    main()
