"""Seeded synthetic workloads shared by the tests, the benchmark and smoke().

This module holds problem descriptions and input arrays only: grid sizes,
operator parameters, initial conditions, forcing vectors and the seeded
random draws of the batched workload.  It contains none of the method's
arithmetic (no quadrature, no matrices, no time stepping) and imports
neither the oracle nor the HIP library, so both sides can consume it.

Domains follow the problem statement: 1D problems live on [-1, 1], 2D ones
on the unit square, both with zero exterior; the grid has ``n`` interior
points per axis with spacing ``h = (hi - lo)/(n + 1)``.  2D vectors are in
lexicographic order with the first coordinate slowest.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

__all__ = ["Workload", "config1", "config2", "config3", "config4_instances", "serving_pool", "serving_trace", "request_u0",
           "grid_points", "bump_1d", "ball_power", "gaussians_2d", "workload_key", "lshape_mask", "lshape_distance",
           "variable_order_lshape"]


@dataclass
class Workload:
    name: str
    dim: int
    n: int
    lo: float
    hi: float
    s: float
    lam: float = 0.0
    C: float | None = None           # None: the fractional-Laplacian constant c_{d,s}
    a: float = 0.0                   # diffusion coefficient (sigma^2 / 2)
    b: tuple = (0.0, 0.0)            # drift
    c: float = 0.0                   # killing rate (<= 0)
    r0: float = 0.2                  # singular-window radius
    dt: float = 1e-3
    steps: int = 100
    leaf: int = 64
    eta: float = 1.0
    n_block: int = 4
    aca_tol: float = 1e-10
    max_rank: int = 32
    lu_tol: float = 1e-12
    u0: np.ndarray | None = None
    g: np.ndarray | None = None      # spatial forcing profile (f(x,t) = phi(t) g(x))
    phi: np.ndarray | None = None    # phi at t_0 .. t_steps
    extra: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.n if self.dim == 1 else self.n * self.n

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


def grid_points(dim: int, n: int, lo: float, hi: float) -> np.ndarray:
    h = (hi - lo) / (n + 1)
    x1 = lo + h * np.arange(1, n + 1, dtype=np.float64)
    if dim == 1:
        return x1[:, None]
    X, Y = np.meshgrid(x1, x1, indexing="ij")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def ball_power(x: np.ndarray, s: float) -> np.ndarray:
    """(1 - |x|^2)_+^s."""
    r2 = (x * x).sum(axis=1)
    return np.maximum(1.0 - r2, 0.0) ** s


def bump_1d(x: np.ndarray, std: float = 0.1) -> np.ndarray:
    """Unit-peak Gaussian bump, mean 0."""
    return np.exp(-x[:, 0] ** 2 / (2.0 * std * std))


def gaussians_2d(x: np.ndarray, seed: int, count: int = 8, std: float = 0.05):
    """Sum of ``count`` Gaussians, centres U([0.2,0.8]^2) then amplitudes U(0,1)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(0.2, 0.8, size=(count, 2))
    amps = rng.uniform(0.0, 1.0, size=count)
    u = np.zeros(x.shape[0])
    for cj, aj in zip(centres, amps):
        d2 = ((x - cj) ** 2).sum(axis=1)
        u += aj * np.exp(-d2 / (2.0 * std * std))
    return u


def _ball_forcing_constant(d: int, s: float) -> float:
    # closed-form value of (-Delta)^s (1-|x|^2)_+^s on the ball: it is the
    # problem statement's forcing amplitude, not something the solver derives
    return 4.0 ** s * math.gamma(1.0 + s) * math.gamma(d / 2.0 + s) / math.gamma(d / 2.0)


def config1(n: int = 1024, steps: int = 100) -> Workload:
    """1D fractional Laplacian, s = 0.5, N = 1024, dt = 1e-3, 100 steps, FP64;
    u0 = (1 - x^2)_+^s, forcing K e^{-t} with K the ball constant."""
    w = Workload(name="frac1d_s0.5_n%d" % n, dim=1, n=n, lo=-1.0, hi=1.0, s=0.5,
                 dt=1e-3, steps=steps, aca_tol=1e-10, lu_tol=1e-12)
    x = grid_points(1, n, w.lo, w.hi)
    w.u0 = ball_power(x, w.s)
    K = _ball_forcing_constant(1, w.s)
    w.g = np.full(n, K)
    w.phi = np.exp(-w.dt * np.arange(steps + 1))
    return w


def config2(n: int = 65536, steps: int = 1000) -> Workload:
    """1D full Levy generator: tempered-stable jumps s = 0.75, lambda = 1,
    drift 0.5, sigma^2 = 0.1 (a = sigma^2/2), dt = 1e-4, 1000 steps,
    Gaussian bump u0 with std 0.1."""
    w = Workload(name="tempered1d_s0.75_n%d" % n, dim=1, n=n, lo=-1.0, hi=1.0,
                 s=0.75, lam=1.0, a=0.05, b=(0.5, 0.0), c=0.0, dt=1e-4,
                 steps=steps, aca_tol=1e-10, lu_tol=1e-12)
    x = grid_points(1, n, w.lo, w.hi)
    w.u0 = bump_1d(x, 0.1)
    return w


def config3(s: float = 0.75, n: int = 256, steps: int = 200, seed: int = 1812) -> Workload:
    """2D fractional Laplacian on the unit square, n x n grid, dt = 1e-3,
    200 steps, ACA rank <= 32 at 1e-8, seeded 8-Gaussian u0."""
    w = Workload(name="frac2d_s%g_%dx%d" % (s, n, n), dim=2, n=n, lo=0.0, hi=1.0,
                 s=s, dt=1e-3, steps=steps, aca_tol=1e-8, max_rank=32,
                 lu_tol=1e-10)
    x = grid_points(2, n, w.lo, w.hi)
    w.u0 = gaussians_2d(x, seed)
    return w


def steady_poisson(n: int = 65536, s: float = 0.5, dt: float = 1e4) -> Workload:
    """Steady fractional Poisson problem (-Delta)^s u = 1 on [-1, 1] with
    zero exterior (Sec. 5.3): right-hand side f = 1 (kept in ``g``); the
    preconditioning factor is that of I - dt/2 G with dt = 1e4 (far above
    1/lambda_min of -G, so the factor is nearly proportional to -G)."""
    w = Workload(name="frac_poisson1d_s%g_n%d" % (s, n), dim=1, n=n, lo=-1.0, hi=1.0, s=s, dt=dt,
                 steps=0, aca_tol=1e-10, max_rank=16, lu_tol=1e-6)
    w.g = np.ones(n)
    return w


def lshape_mask(n: int) -> np.ndarray:
    """Grid points of the L-shaped domain [-1, 1]^2 without [0, 1]^2 (Sec. 5.4)
    on the n x n interior grid of [-1, 1]^2: True where the point is not in
    the removed quadrant (x1 >= 0 and x2 >= 0).  Even n puts no grid point on
    the two inner edges, so N = 3 n^2 / 4 (675, 1200, 2700, 4800, 7500 for
    n = 30, 40, 60, 80, 100: the sizes the paper reports)."""
    x = grid_points(2, n, -1.0, 1.0)
    return ~((x[:, 0] >= 0.0) & (x[:, 1] >= 0.0)).reshape(n, n)


def _segment_distance(x: np.ndarray, a, b) -> np.ndarray:
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    ab = b - a
    t = np.clip(((x - a) @ ab) / (ab @ ab), 0.0, 1.0)
    return np.linalg.norm(x - (a + t[:, None] * ab), axis=1)


def lshape_distance(x: np.ndarray) -> np.ndarray:
    """Distance d(x) of points of the L-shaped domain to its boundary: the
    outer square's four sides and the inner edges {0} x [0, 1] and
    [0, 1] x {0}."""
    outer = np.minimum.reduce([1.0 - x[:, 0], 1.0 + x[:, 0], 1.0 - x[:, 1], 1.0 + x[:, 1]])
    inner = np.minimum(_segment_distance(x, (0.0, 0.0), (0.0, 1.0)), _segment_distance(x, (0.0, 0.0), (1.0, 0.0)))
    return np.minimum(outer, inner)


def variable_order_lshape(n: int = 100) -> dict:
    """The variable-order fractional Poisson problem of Sec. 5.4
    (eq. equ:2dmodel): -(-Delta)^{s(x)} u = f on the L-shaped domain, u = 0
    outside; s(x) = 0.9 - 0.8 d(x); f the sum of three Gaussians
    exp(-10 |x - x_k|^2) at (-0.5, 0.5), (0.5, -0.5), (-0.5, -0.5).  The
    paper's tolerances: eps1 = 1e-4 for the construction (aca_tol), eps2 =
    1e-10 for the H-LU (lu_tol).  Returns the mask, the points of the
    unknowns (grid order), s and f on them."""
    mask = lshape_mask(n)
    x = grid_points(2, n, -1.0, 1.0)[mask.reshape(-1)]
    s = 0.9 - 0.8 * lshape_distance(x)
    f = np.zeros(len(x))
    for c in ((-0.5, 0.5), (0.5, -0.5), (-0.5, -0.5)):
        f += np.exp(-10.0 * ((x - np.asarray(c)) ** 2).sum(axis=1))
    return {"name": "varorder_lshape_n%d" % n, "n": n, "N": int(mask.sum()), "mask": mask, "x": x, "s": s,
            "f": f, "aca_tol": 1e-4, "lu_tol": 1e-10}


def config4_instances(count: int = 512, seed: int = 8324, nmin_log2: float = 10.0,
                      nmax_log2: float = 15.0, steps: int = 100) -> list:
    """Independent 1D tempered instances: N log-uniform, s ~ U(0.1, 0.9),
    drift ~ U(-1, 1), sigma^2 ~ U(0, 0.2), lambda ~ U(0, 2); Gaussian-bump u0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(round(2.0 ** rng.uniform(nmin_log2, nmax_log2)))
        s = float(rng.uniform(0.1, 0.9))
        b = float(rng.uniform(-1.0, 1.0))
        sig2 = float(rng.uniform(0.0, 0.2))
        lam = float(rng.uniform(0.0, 2.0))
        w = Workload(name="inst%d" % i, dim=1, n=n, lo=-1.0, hi=1.0, s=s, lam=lam,
                     a=0.5 * sig2, b=(b, 0.0), dt=1e-3, steps=steps,
                     aca_tol=1e-10, lu_tol=1e-12)
        w.u0 = bump_1d(grid_points(1, n, -1.0, 1.0), 0.1)
        out.append(w)
    return out


def serving_pool(seed: int = 356, size: int = 64, n1d_log2=(12.0, 16.0), side=(64, 256)) -> dict:
    """Operator configurations requests draw from (so that parameter sets
    repeat): `size` 1D tempered problems (N log-uniform, s, drift, sigma^2,
    lambda as in the batched workload) and `size` 2D tempered problems on the
    unit square (side uniform in [side[0], side[1]]; s, lambda, sigma^2 as in
    the batched workload, each drift component ~ U(-1, 1); ACA at 1e-8 with
    rank <= 32).  Returns {"1d": [...], "2d": [...]}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p1, p2 = [], []
    for i in range(size):
        n = int(round(2.0 ** rng.uniform(*n1d_log2)))
        s = float(rng.uniform(0.1, 0.9))
        b = float(rng.uniform(-1.0, 1.0))
        sig2 = float(rng.uniform(0.0, 0.2))
        lam = float(rng.uniform(0.0, 2.0))
        p1.append(Workload(name="pool1d_%d" % i, dim=1, n=n, lo=-1.0, hi=1.0, s=s, lam=lam, a=0.5 * sig2,
                           b=(b, 0.0), dt=1e-3, aca_tol=1e-10, max_rank=16, lu_tol=1e-6))
    for i in range(size):
        n = int(rng.integers(side[0], side[1] + 1))
        s = float(rng.uniform(0.1, 0.9))
        b = (float(rng.uniform(-1.0, 1.0)), float(rng.uniform(-1.0, 1.0)))
        sig2 = float(rng.uniform(0.0, 0.2))
        lam = float(rng.uniform(0.0, 2.0))
        p2.append(Workload(name="pool2d_%d" % i, dim=2, n=n, lo=0.0, hi=1.0, s=s, lam=lam, a=0.5 * sig2, b=b,
                           dt=1e-3, aca_tol=1e-8, max_rank=32, lu_tol=1e-6))
    return {"1d": p1, "2d": p2}


def serving_trace(rate: float = 200.0, duration: float = 60.0, seed: int = 355, frac_1d: float = 0.7,
                  horizon=(50, 500), pool: dict | None = None) -> list:
    """Poisson arrivals (exponential gaps of mean 1/rate) over `duration`
    seconds; each request picks 1D with probability frac_1d, a pool entry
    uniformly and a horizon uniform in [horizon[0], horizon[1]] steps.
    Returns dicts {"t": arrival time, "w": Workload (without u0), "steps":
    horizon, "seed": the request's seed}; request_u0() makes its u0."""
    pool = pool if pool is not None else serving_pool()
    rng = np.random.Generator(np.random.PCG64(seed))
    out, t = [], 0.0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t > duration:
            break
        one_d = bool(rng.uniform() < frac_1d)
        lst = pool["1d"] if one_d else pool["2d"]
        w = lst[int(rng.integers(0, len(lst)))]
        steps = int(rng.integers(horizon[0], horizon[1] + 1))
        rseed = int(rng.integers(0, 2 ** 31 - 1))
        out.append({"t": t, "w": w.with_(steps=steps), "steps": steps, "seed": rseed})
    return out


def request_u0(req: dict) -> np.ndarray:
    """Initial condition of a serving request: 1D the Gaussian bump, 2D eight
    Gaussians drawn with the request's seed."""
    w = req["w"]
    x = grid_points(w.dim, w.n, w.lo, w.hi)
    return bump_1d(x, 0.1) if w.dim == 1 else gaussians_2d(x, req["seed"])


def workload_key(w: Workload) -> str:
    """A hash of everything that fixes a workload's CN trajectory: the problem
    parameters, the step size and count, and the bytes of u0, g and phi.
    Stored results are keyed by it, so a changed recipe cannot be compared
    with a result made for the old one."""
    import hashlib
    import json
    h = hashlib.sha256()
    scal = {k: getattr(w, k) for k in ("dim", "n", "lo", "hi", "s", "lam", "C", "a", "c", "r0", "dt", "steps")}
    scal["b"] = list(w.b)
    h.update(json.dumps(scal, sort_keys=True).encode())
    for arr in (w.u0, w.g, w.phi):
        h.update(b"-" if arr is None else np.ascontiguousarray(arr, dtype=np.float64).tobytes())
    return h.hexdigest()[:16]
