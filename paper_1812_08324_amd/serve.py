"""Replay of a request trace through the library's serving loop
(hlevy_server_*), with arrival-to-result latencies on the host clock.

Requests are submitted when the host clock passes their arrival time; the
loop polls scheduling rounds (admission, joint factorisation of operators
not in the cache, one batched chunk of steps for all active requests) until
every request has finished.  All work runs in the HIP library; this module
only keeps time and moves vectors.
"""
from __future__ import annotations

import time

import numpy as np


def _problem(H, w):
    p = H.make_problem(w.dim, w.n, w.lo, w.hi, w.s, lam=w.lam, C_=w.C, a=w.a, b=w.b, c=w.c, r0=w.r0)
    hp = H.make_hparams(leaf=w.leaf, eta=w.eta, n_block=w.n_block, aca_tol=w.aca_tol, max_rank=w.max_rank)
    return p, hp


def replay(H, torch, trace, make_u0, keep_outputs=False, realtime=True, log=None, **server_kw) -> dict:
    """Serve `trace` (dicts with "t", "w", "steps") on a new Server.

    make_u0(req) -> numpy initial condition.  realtime=False submits every
    request at time 0 (a closed batch).  Returns latencies (s) per request,
    p50 / p99, throughput and the server's counters; with keep_outputs the
    result vectors (device tensors) by request index."""
    srv = H.Server(**server_kw)
    n = len(trace)
    arrival = np.array([r["t"] if realtime else 0.0 for r in trace])
    done_at = np.full(n, np.nan)
    outs = {}
    id2idx = {}
    # initial conditions are made ahead of the clock (host work, not serving)
    u0s = [torch.tensor(make_u0(r), dtype=torch.float64, device="cuda") for r in trace]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nxt = 0
    finished = 0
    last_log = 0.0
    while finished < n:
        if log is not None and time.perf_counter() - t0 - last_log > 5.0:
            last_log = time.perf_counter() - t0
            log(f"serving: {finished}/{n} done, {nxt} submitted at t={last_log:.1f}s")
        now = time.perf_counter() - t0
        while nxt < n and arrival[nxt] <= now:
            r = trace[nxt]
            p, hp = _problem(H, r["w"])
            out = torch.empty_like(u0s[nxt])
            rid = srv.submit(p, hp, r["w"].dt, r["steps"], u0s[nxt], out)
            id2idx[rid] = nxt
            if keep_outputs:
                outs[nxt] = out
            u0s[nxt] = None
            nxt += 1
        st = srv.stats()
        if st["active"] == 0 and st["queued"] == 0:
            if nxt < n:
                time.sleep(max(0.0, arrival[nxt] - (time.perf_counter() - t0)))
            continue
        for rid in srv.poll():
            done_at[id2idx[rid]] = time.perf_counter() - t0
            finished += 1
    wall = time.perf_counter() - t0
    lat = done_at - arrival
    st = srv.stats()
    steps = sum(r["steps"] for r in trace)
    res = {
        "requests": n,
        "wall_s": wall,
        "latency_p50_s": float(np.percentile(lat, 50)),
        "latency_p99_s": float(np.percentile(lat, 99)),
        "latency_mean_s": float(lat.mean()),
        "problem_steps": steps,
        "problem_steps_per_s": steps / wall,
        "requests_per_s": n / wall,
        "cache_hit_rate": st["cache_hits"] / max(1, st["cache_hits"] + st["cache_misses"]),
        "server": st,
        "latencies": lat,
    }
    if keep_outputs:
        res["outputs"] = outs
    del srv
    return res
