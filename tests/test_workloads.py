"""CPU tests of the seeded input recipes (workloads/): every generator is
deterministic for its seed and draws the shapes and parameter ranges the
measurements are quoted on (the batched instances, the serving pool and
trace, the 2D initial condition)."""
import numpy as np
import pytest

import workloads as W


def test_batched_instances_deterministic_and_in_range():
    a = W.config4_instances()
    b = W.config4_instances()
    assert len(a) == 512
    assert [w.n for w in a] == [w.n for w in b]
    assert all(np.array_equal(x.u0, y.u0) for x, y in zip(a[:8], b[:8]))
    n = np.array([w.n for w in a])
    assert n.min() >= 2 ** 10 and n.max() <= 2 ** 15
    # N log-uniform on [2^10, 2^15]: the median sits near 2^12.5
    assert 2 ** 12.2 < np.median(n) < 2 ** 12.8
    for w in a:
        assert 0.1 <= w.s <= 0.9 and 0.0 <= w.lam <= 2.0 and -1.0 <= w.b[0] <= 1.0
        assert 0.0 <= 2 * w.a <= 0.2
        assert w.steps == 100 and w.dt == 1e-3 and w.u0.shape == (w.n,)
    assert W.config4_instances(seed=8325)[0].n != a[0].n or W.config4_instances(seed=8325)[0].s != a[0].s


def test_serving_trace_deterministic_and_poisson():
    pool = W.serving_pool()
    assert len(pool["1d"]) == 64 and len(pool["2d"]) == 64
    tr = W.serving_trace(pool=pool)
    tr2 = W.serving_trace(pool=pool)
    assert [r["t"] for r in tr] == [r["t"] for r in tr2]
    # rate 200/s over 60 s: about 12000 arrivals (Poisson: sd ~ 110)
    assert 11500 < len(tr) < 12500
    t = np.array([r["t"] for r in tr])
    assert np.all(np.diff(t) > 0) and t[-1] <= 60.0
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 200) < 2e-4
    frac_1d = np.mean([r["w"].dim == 1 for r in tr])
    assert 0.68 < frac_1d < 0.72
    h = np.array([r["steps"] for r in tr])
    assert h.min() >= 50 and h.max() <= 500
    # parameter sets repeat: every request's operator comes from the pool
    names = {w.name for w in pool["1d"] + pool["2d"]}
    assert all(r["w"].name in names for r in tr)
    # 2D operators take the batched workload's parameter ranges
    p2 = pool["2d"]
    assert all(64 <= w.n <= 256 and 0.1 <= w.s <= 0.9 and 0.0 <= w.lam <= 2.0 and 0.0 <= w.a <= 0.1
               and abs(w.b[0]) <= 1.0 and abs(w.b[1]) <= 1.0 for w in p2)
    assert len({w.lam for w in p2}) == 64 and len({w.b[1] for w in p2}) == 64


def test_serving_request_u0_seeded():
    tr = W.serving_trace(duration=0.5, frac_1d=0.0)
    assert tr, "a 0.5 s window at 200/s has arrivals"
    r = tr[0]
    u = W.request_u0(r)
    assert u.shape == (r["w"].n ** 2,)
    assert np.array_equal(u, W.request_u0(r))
    other = dict(r, seed=r["seed"] + 1)
    assert not np.array_equal(u, W.request_u0(other))


def test_config3_initial_condition():
    w = W.config3()
    assert w.N == 256 * 256 and w.max_rank == 32 and w.aca_tol == 1e-8
    assert np.array_equal(w.u0, W.config3().u0)
    # eight Gaussians of std 0.05 with centres in [0.2, 0.8]^2 and amplitudes
    # in (0, 1): the field is positive, at most 8, and small at the corners
    assert w.u0.min() >= 0.0 and 0.0 < w.u0.max() <= 8.0
    u = w.u0.reshape(256, 256)
    assert max(u[0, 0], u[0, -1], u[-1, 0], u[-1, -1]) < 1e-6


def test_config1_forcing_and_initial_condition():
    w = W.config1()
    x = W.grid_points(1, w.n, w.lo, w.hi)[:, 0]   # points as an (N, 1) array
    assert np.allclose(w.u0, np.sqrt(np.clip(1 - x ** 2, 0, None)))
    assert np.all(w.g == w.g[0]) and w.g[0] > 0
    assert np.allclose(w.phi, np.exp(-w.dt * np.arange(w.steps + 1)))
