"""Writes the oracle's CN results at the benchmark sizes into this folder.

Calls only ``oracle/`` (the memory-lean dense CN of ``cn_run_lean``) and the
seeded input recipes of ``workloads``.  The LU goes through MKL (torch's CPU
LAPACK, threads from OMP_NUM_THREADS), the step loop's triangular products
and solves through scipy's OpenBLAS (OPENBLAS_NUM_THREADS); the runs stored
here used 6 threads each on an 8-core host.  Each result is ``<name>.npz`` (u at
the final step and the per-step 2-norms) plus ``<name>.json`` (the workload
key, the oracle's assembly, factorisation and stepping times, and the host
they were measured on).  One N = 65536 run holds one 34 GB array.

    python tests/golden/make_fullsize_goldens.py tempered1d_s0.75_n65536 \
        frac2d_s0.75_256x256 frac2d_s0.25_256x256
"""
import json
import os
import platform
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W                                   # noqa: E402
from oracle.levy_oracle import Problem, cn_run_lean     # noqa: E402

RECIPES = {
    "tempered1d_s0.75_n65536": lambda: W.config2(),
    "tempered1d_s0.75_n16384": lambda: W.config2(n=16384),
    "frac2d_s0.75_256x256": lambda: W.config3(0.75),
    "frac2d_s0.25_256x256": lambda: W.config3(0.25),
}


def oracle_problem(w):
    return Problem(dim=w.dim, n=w.n, lo=w.lo, hi=w.hi, a=w.a, b=tuple(w.b), c=w.c, s=w.s,
                   lam=w.lam, C=w.C, r0=w.r0)


def host_info():
    info = {"nproc": os.cpu_count(), "machine": platform.machine()}
    try:
        with open("/proc/cpuinfo") as f:
            info["cpu"] = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
        with open("/proc/meminfo") as f:
            info["mem_kib"] = int(next(l.split()[1] for l in f if l.startswith("MemTotal")))
    except (OSError, StopIteration):
        pass
    try:
        cfg = np.show_config(mode="dicts")
        blas = cfg["Build Dependencies"]["blas"]
        info["blas"] = f'{blas.get("name")} {blas.get("version")}'
    except Exception:
        pass
    info["blas_threads"] = os.environ.get("OPENBLAS_NUM_THREADS", "default (all cores)")
    try:
        import torch
        info["lu_lapack"] = f"MKL getrf through torch {torch.__version__}, {torch.get_num_threads()} threads"
    except Exception:
        pass
    return info


def make(name):
    w = RECIPES[name]()
    key = W.workload_key(w)

    def log(msg):
        print(f"[{name} {time.strftime('%H:%M:%S')}] {msg}", flush=True)

    log(f"N={w.N} steps={w.steps} dt={w.dt} key={key}")
    res = cn_run_lean(oracle_problem(w), w.dt, w.steps, w.u0, w.g, w.phi, keep_norms=True, log=log)
    np.savez(os.path.join(HERE, name + ".npz"), u=res.u, norms=np.asarray(res.norms))
    meta = {"name": name, "key": key, "N": w.N, "steps": w.steps, "dt": w.dt,
            "timings": res.timings, "steps_per_s": w.steps / res.timings["steps_s"],
            "host": host_info(),
            "command": "python tests/golden/make_fullsize_goldens.py " + name}
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(meta, f, indent=1)
    log(f"done {res.timings}")


if __name__ == "__main__":
    for nm in sys.argv[1:]:
        make(nm)
