"""GPU parity at the sizes the benchmark runs (through the C ABI).

The full CN trajectories of the N = 65536 tempered workload (1000 steps)
and of the 256 x 256 fractional workloads (s = 0.75 and 0.25, 200 steps)
are compared with the dense oracle's, computed once on the CPU by
tests/golden/make_fullsize_goldens.py (a single N x N array factored in
place) and stored there with the hash of the workload they belong to.  The
operator is also compared with oracle rows, and the solves through the
residual of M x = b measured with that operator.  The trajectory at
N = 4096 is compared with the dense oracle computed here.
"""
import json
import os

import numpy as np
import pytest

from oracle.levy_oracle import Problem, cn_run, generator_dense, generator_row, quadrature_constants
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_08324_amd import hlevy
    return hlevy


def oracle_problem(w):
    return Problem(dim=w.dim, n=w.n, lo=w.lo, hi=w.hi, a=w.a, b=tuple(w.b), c=w.c, s=w.s,
                   lam=w.lam, C=w.C, r0=w.r0)


def lib(H, w, max_rank=16):
    p = H.make_problem(w.dim, w.n, w.lo, w.hi, w.s, lam=w.lam, C_=w.C, a=w.a, b=w.b, c=w.c, r0=w.r0)
    hp = H.make_hparams(leaf=w.leaf, eta=w.eta, n_block=w.n_block, aca_tol=w.aca_tol, max_rank=max_rank)
    return p, hp


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name, w):
    """u at the last step from the stored full-size oracle run `name`, after
    checking that it was made for this workload (same hash)."""
    path = os.path.join(GOLDEN, name + ".npz")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle result {name} (tests/golden/make_fullsize_goldens.py writes it)")
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        meta = json.load(f)
    assert meta["key"] == W.workload_key(w), "stored oracle result made for another workload"
    with np.load(path) as z:
        return z["u"]


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def full(H):
    """The N = 65536 tempered workload: operator, FP64 and mixed factors."""
    w = W.config2()
    p, hp = lib(H, w)
    op = H.assemble(p, hp)
    f64 = H.factor(op, w.dt, H.PREC_FP64, 1e-12)
    fmx = H.factor(op, w.dt, H.PREC_MIXED, 1e-6)
    return w, op, f64, fmx


def residual(H, w, op, x, b):
    y = torch.empty_like(x)
    H.matvec(op, x, y)
    r = b - (x - 0.5 * w.dt * y)
    return float(torch.linalg.norm(r) / torch.linalg.norm(b))


def test_operator_rows_at_full_size(H, full):
    """y = G x at N = 65536 against oracle rows (sampled, boundaries included),
    |y_i - g_i . x| <= 10 aca_tol |g_i| |x|.  The 1/h^2 near field dominates
    this bound; the far field is held to the ACA tolerance block by block
    in test_gpu_far_field.py."""
    w, op, _, _ = full
    rng = np.random.Generator(np.random.PCG64(65536))
    x = rng.standard_normal(w.N)
    y = torch.empty(w.N, dtype=torch.float64, device="cuda")
    H.matvec(op, dev(x), y)
    y = host(y)
    p = oracle_problem(w)
    consts = quadrature_constants(p)
    rows = np.unique(np.concatenate([[0, 1, 63, 64, w.N // 2, w.N - 65, w.N - 2, w.N - 1],
                                     rng.integers(0, w.N, 40)]))
    nx = np.linalg.norm(x)
    for i in rows:
        g = generator_row(p, int(i), consts)
        ref = float(g @ x)
        assert abs(y[i] - ref) <= 10 * w.aca_tol * np.linalg.norm(g) * nx, (int(i), y[i], ref)


@pytest.mark.parametrize("kind", ["smooth", "random"])
def test_fp64_solve_residual_at_full_size(H, full, kind):
    """FP64 factors with the default refinement sweep: relative residual of
    M x = b at N = 65536 below 1e-10."""
    w, op, f64, _ = full
    if kind == "smooth":
        b = dev(w.u0)
    else:
        b = dev(np.random.Generator(np.random.PCG64(7)).standard_normal(w.N))
    x = torch.empty_like(b)
    H.solve(f64, b, x)
    assert residual(H, w, op, x, b) < 1e-10


def test_mixed_solve_residual_at_full_size(H, full):
    """Mixed factors (FP32 inverse factors at 1e-6): the preconditioner alone
    is near 1e-5, one FP64 refinement sweep brings the residual below 1e-9."""
    w, op, _, fmx = full
    b = dev(np.random.Generator(np.random.PCG64(8)).standard_normal(w.N))
    x = torch.empty_like(b)
    res = []
    for sweeps in (0, 1, 2):
        H.solve(fmx, b, x, refine={"sweeps": sweeps})
        res.append(residual(H, w, op, x, b))
    assert res[0] < 1e-4, res
    assert res[1] < 1e-9 and res[2] < 1e-9, res


# FP64 agreement bound of two correct implementations of the recursion at
# this size.  The generator's diagonal is of size 1/h^2 (1.3e8 here), and one
# ulp of difference in each diagonal entry moves the 1000-step trajectory by
# 3.1e-12 at N = 4096 and 5.6e-11 at N = 16384 (measured with the oracle,
# tests/test_fp64_floor.py), about 1e-9 at N = 65536.  Diagonals summed in
# another order differ by a few ulps, so two FP64 implementations agree to a
# few 1e-9 here (the GPU's FP64 path: 5.3e-9, the same for ACA tolerances
# 1e-10 to 1e-13 and one or two sweeps), while at N = 16384 the FP64 path
# meets 1e-10.
FP64_BAR_FULL = 1e-8


@pytest.mark.parametrize("path", ["fp64_plain", "fp64", "mixed"])
def test_trajectory_vs_fullsize_oracle(H, full, path):
    """1000 CN steps at N = 65536 against the dense oracle's trajectory:
    the FP64 direct H-solve (no refinement) and with one refinement sweep
    within the FP64 agreement bound FP64_BAR_FULL, the mixed path (one
    sweep per step) within 1e-8."""
    w, op, f64, fmx = full
    ref = golden("tempered1d_s0.75_n65536", w)
    fac, sweeps, bar = {"fp64_plain": (f64, 0, FP64_BAR_FULL), "fp64": (f64, 1, FP64_BAR_FULL),
                        "mixed": (fmx, 1, 1e-8)}[path]
    u = dev(w.u0)
    st = H.step(fac, u, w.steps, refine={"sweeps": sweeps}, stats=True)
    err = rel(host(u), ref)
    print(f"{path}: rel-L2 vs oracle {err:.3e}, last residual {st['last_rel_residual']:.2e}")
    assert err <= bar, err
    assert st["rank_overflows"] == 0


def test_fp64_trajectory_vs_oracle_n16384(H):
    """1000 CN steps of the tempered workload at N = 16384 (the headline
    operator parameters, dt = 1e-4): the FP64 path within 1e-10 of the
    stored dense oracle trajectory."""
    w = W.config2(n=16384, steps=1000)
    ref = golden("tempered1d_s0.75_n16384", w)
    p, hp = lib(H, w)
    op = H.assemble(p, hp)
    f64 = H.factor(op, w.dt, H.PREC_FP64, 1e-12)
    u = dev(w.u0)
    H.step(f64, u, w.steps, refine={"sweeps": 1})
    err = rel(host(u), ref)
    print(f"N = 16384 FP64 vs oracle {err:.3e}")
    assert err <= 1e-10, err


def test_tempered_trajectory_vs_oracle_n4096(H):
    """The tempered workload's operator at N = 4096, 200 CN steps: FP64 path
    within 1e-10, mixed path (FP32 inverse factors, one sweep) and BF16 path
    (BF16 low-rank leaves, two sweeps) within 1e-8 of the dense oracle."""
    w = W.config2(n=4096, steps=200)
    p, hp = lib(H, w)
    op = H.assemble(p, hp)
    ref = cn_run(generator_dense(oracle_problem(w)), w.dt, w.steps, w.u0).u
    nref = np.linalg.norm(ref)
    f64 = H.factor(op, w.dt, H.PREC_FP64, 1e-12)
    u = dev(w.u0)
    H.step(f64, u, w.steps)
    e64 = np.linalg.norm(host(u) - ref) / nref
    fmx = H.factor(op, w.dt, H.PREC_MIXED, 1e-6)
    u = dev(w.u0)
    H.step(fmx, u, w.steps, refine={"sweeps": 1})
    emx = np.linalg.norm(host(u) - ref) / nref
    # BF16 low-rank leaves of the inverse factors: a coarser preconditioner,
    # two sweeps per step
    fbf = H.factor(op, w.dt, H.PREC_MIXED_BF16, 1e-6)
    u = dev(w.u0)
    H.step(fbf, u, w.steps, refine={"sweeps": 2})
    ebf = np.linalg.norm(host(u) - ref) / nref
    assert e64 <= 1e-10, e64
    assert emx <= 1e-8, emx
    assert ebf <= 1e-8, ebf
    fi, fb = H.fac_info(fmx), H.fac_info(fbf)
    assert fb["product_bytes"][1] < fi["product_bytes"][1] and fb["product_bytes"][2] < fi["product_bytes"][2]


@pytest.fixture(scope="module", params=[0.75, 0.25], ids=["s0.75", "s0.25"])
def full2d(H, request):
    """The 2D workload at full size: 256 x 256 grid, s = 0.75 and 0.25, ACA
    rank <= 32 at 1e-8; FP64 factors (lu_tol 1e-10) and mixed factors (1e-6)."""
    w = W.config3(s=request.param, n=256)
    p, hp = lib(H, w, max_rank=w.max_rank)
    op = H.assemble(p, hp)
    assert H.op_info(op)["rank_overflows"] == 0
    f64 = H.factor(op, w.dt, H.PREC_FP64, w.lu_tol)
    fmx = H.factor(op, w.dt, H.PREC_MIXED, 1e-6)
    return w, op, f64, fmx


def test_2d_operator_rows_at_full_size(H, full2d):
    """y = G x on the 256 x 256 grid against oracle rows (sampled: corners,
    edges, centre and seeded interior points), each within 10 aca_tol
    |g_i| |x|."""
    w, op, _, _ = full2d
    rng = np.random.Generator(np.random.PCG64(256))
    x = rng.standard_normal(w.N)
    y = torch.empty(w.N, dtype=torch.float64, device="cuda")
    H.matvec(op, dev(x), y)
    y = host(y)
    p = oracle_problem(w)
    consts = quadrature_constants(p)
    n = w.n
    rows = np.unique(np.concatenate([[0, n - 1, n * (n - 1), w.N - 1, n // 2, n * (n // 2) + n // 2,
                                      n * 17 + 1], rng.integers(0, w.N, 25)]))
    nx = np.linalg.norm(x)
    for i in rows:
        g = generator_row(p, int(i), consts)
        ref = float(g @ x)
        assert abs(y[i] - ref) <= 10 * w.aca_tol * np.linalg.norm(g) * nx, (int(i), y[i], ref)


def test_2d_solve_residuals_at_full_size(H, full2d):
    """M x = b on the 256 x 256 grid: FP64 factors (one default sweep) and
    mixed factors (one sweep) both below 1e-10 relative residual."""
    w, op, f64, fmx = full2d
    b = dev(np.random.Generator(np.random.PCG64(9)).standard_normal(w.N))
    x = torch.empty_like(b)
    H.solve(f64, b, x)
    assert residual(H, w, op, x, b) < 1e-10
    H.solve(fmx, b, x, refine={"sweeps": 1})
    assert residual(H, w, op, x, b) < 1e-10


def test_2d_trajectories_vs_fullsize_oracle(H, full2d):
    """200 CN steps on the 256 x 256 grid against the dense oracle's
    trajectory: the FP64 path (one sweep: its factors overflow the rank
    capacity, which the sweep repairs) within 1e-10, the mixed path (one
    sweep) within 1e-8."""
    w, op, f64, fmx = full2d
    ref = golden(w.name, w)
    ua = dev(w.u0)
    ub = dev(w.u0)
    H.step(f64, ua, w.steps, refine={"sweeps": 1})
    H.step(fmx, ub, w.steps, refine={"sweeps": 1})
    e64, emx = rel(host(ua), ref), rel(host(ub), ref)
    print(f"{w.name}: FP64 {e64:.3e}, mixed {emx:.3e} (FP64 factor overflows "
          f"{H.fac_info(f64)['rank_overflows']})")
    assert e64 <= 1e-10, e64
    assert emx <= 1e-8, emx
