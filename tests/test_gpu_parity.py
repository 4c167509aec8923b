"""GPU parity of the HIP path (through the C ABI) against the CPU oracle on
the same seeded inputs."""
import math

import numpy as np
import pytest

from oracle.levy_oracle import Problem, cn_run, generator_dense, quadrature_constants
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


def lib_problem(H, w):
    return H.make_problem(w.dim, w.n, w.lo, w.hi, w.s, lam=w.lam, C_=w.C, a=w.a, b=w.b, c=w.c, r0=w.r0)


def lib_hparams(H, w):
    return H.make_hparams(leaf=w.leaf, eta=w.eta, n_block=w.n_block, aca_tol=w.aca_tol,
                          max_rank=w.max_rank if w.dim == 2 else 16)


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


SMALL = {
    "frac1d_s0.5_n1024": lambda: W.config1(),
    "tempered1d_n2000": lambda: W.config2(n=2000, steps=50),
    "frac2d_s0.25_40x40": lambda: W.config3(s=0.25, n=40, steps=20),
    "frac2d_s0.75_33x33": lambda: W.config3(s=0.75, n=33, steps=20),
}


@pytest.mark.parametrize("name", list(SMALL))
def test_constants_match_oracle(H, name):
    w = SMALL[name]()
    op = H.assemble(lib_problem(H, w), lib_hparams(H, w))
    got = H.op_constants(op)
    ref = quadrature_constants(oracle_problem(w))
    for g, key in zip(got, ("S0", "S2", "C2", "T")):
        assert g == pytest.approx(ref[key], rel=1e-12, abs=1e-300), key


@pytest.mark.parametrize("name", list(SMALL))
def test_densified_operator_matches_dense_generator(H, name):
    w = SMALL[name]()
    op = H.assemble(lib_problem(H, w), lib_hparams(H, w))
    N = w.N
    dense = torch.zeros(N * N, dtype=torch.float64, device="cuda")
    H.op_densify(op, dense)
    Gh = host(dense).reshape(N, N)
    G = generator_dense(oracle_problem(w))
    err = np.linalg.norm(Gh - G) / np.linalg.norm(G)
    assert err < 10 * w.aca_tol, err
    # the near field (every entry within one grid step) is exact arithmetic
    if w.dim == 1:
        band = np.abs(np.subtract.outer(np.arange(N), np.arange(N))) <= 1
        assert np.allclose(Gh[band], G[band], rtol=1e-13, atol=0)
    info = H.op_info(op)
    assert info["rank_overflows"] == 0


@pytest.mark.parametrize("name", list(SMALL))
def test_matvec_matches_oracle(H, name):
    w = SMALL[name]()
    op = H.assemble(lib_problem(H, w), lib_hparams(H, w))
    rng = np.random.Generator(np.random.PCG64(7))
    x = rng.standard_normal(w.N)
    y = torch.empty(w.N, dtype=torch.float64, device="cuda")
    H.matvec(op, dev(x), y)
    ref = generator_dense(oracle_problem(w)) @ x
    err = np.linalg.norm(host(y) - ref) / np.linalg.norm(ref)
    assert err < 10 * w.aca_tol, err


@pytest.mark.parametrize("name", list(SMALL))
def test_solve_matches_dense_solve(H, name):
    w = SMALL[name]()
    op = H.assemble(lib_problem(H, w), lib_hparams(H, w))
    fac = H.factor(op, w.dt, H.PREC_FP64, w.lu_tol)
    G = generator_dense(oracle_problem(w))
    M = np.eye(w.N) - 0.5 * w.dt * G
    rng = np.random.Generator(np.random.PCG64(11))
    xt = rng.standard_normal(w.N)
    b = M @ xt
    x = torch.empty(w.N, dtype=torch.float64, device="cuda")
    H.solve(fac, dev(b), x)
    err = np.linalg.norm(host(x) - xt) / np.linalg.norm(xt)
    assert err < 1e-9, err


def test_config1_cn_trajectory(H):
    """1D fractional Laplacian s = 1/2, N = 1024, 100 CN steps, FP64:
    relative L2 <= 1e-10 against the dense oracle."""
    w = W.config1()
    op = H.assemble(lib_problem(H, w), lib_hparams(H, w))
    fac = H.factor(op, w.dt, H.PREC_FP64, w.lu_tol)
    u = dev(w.u0)
    g = dev(w.g)
    H.step(fac, u, w.steps, g=g, phi=list(w.phi))
    ref = cn_run(generator_dense(oracle_problem(w)), w.dt, w.steps, w.u0, g=w.g, phi=w.phi).u
    err = np.linalg.norm(host(u) - ref) / np.linalg.norm(ref)
    assert err <= 1e-10, err


@pytest.mark.parametrize("name", ["frac1d_s0.5_n1024", "tempered1d_n2000", "frac2d_s0.75_33x33"])
def test_mixed_solve_with_refinement(H, name):
    """FP32 inverse factors at a loose truncation, FP64 residual refinement:
    two sweeps bring the solve to FP64 accuracy."""
    w = SMALL[name]()
    op = H.assemble(lib_problem(H, w), lib_hparams(H, w))
    fac = H.factor(op, w.dt, H.PREC_MIXED, 1e-6)
    G = generator_dense(oracle_problem(w))
    M = np.eye(w.N) - 0.5 * w.dt * G
    rng = np.random.Generator(np.random.PCG64(13))
    xt = rng.standard_normal(w.N)
    b = M @ xt
    x = torch.empty(w.N, dtype=torch.float64, device="cuda")
    errs = []
    for sweeps in (0, 1, 3):
        H.solve(fac, dev(b), x, refine={"sweeps": sweeps})
        errs.append(np.linalg.norm(host(x) - xt) / np.linalg.norm(xt))
    assert errs[0] < 1e-4, errs
    assert errs[2] < 1e-10, errs
    # refinement converges to the accuracy floor of the H-approximated operator
    assert errs[1] < errs[0] and errs[2] <= 1.01 * errs[1], errs


def test_config1_mixed_trajectory(H):
    """Mixed path on the N = 1024 workload: rel-L2 <= 1e-8 after refinement."""
    w = W.config1()
    op = H.assemble(lib_problem(H, w), lib_hparams(H, w))
    fac = H.factor(op, w.dt, H.PREC_MIXED, 1e-6)
    u = dev(w.u0)
    H.step(fac, u, w.steps, g=dev(w.g), phi=list(w.phi), refine={"sweeps": 2})
    ref = cn_run(generator_dense(oracle_problem(w)), w.dt, w.steps, w.u0, g=w.g, phi=w.phi).u
    err = np.linalg.norm(host(u) - ref) / np.linalg.norm(ref)
    assert err <= 1e-8, err


def test_frac2d_64x64_trajectories():
    """2D fractional Laplacian (s = 0.75) on a 64 x 64 grid, 20 CN steps:
    FP64 path within 1e-10 and mixed path (FP32 inverse factors at 1e-6, two
    refinement sweeps) within 1e-8 of the dense oracle.  The mixed
    factorisation runs rounded additions of up to 64 columns without
    double-double parts."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_08324_amd import hlevy as H
    w = W.config3(s=0.75, n=64, steps=20)
    ref = cn_run(generator_dense(oracle_problem(w)), w.dt, w.steps, w.u0).u
    nref = np.linalg.norm(ref)
    op = H.assemble(lib_problem(H, w), lib_hparams(H, w))
    f64 = H.factor(op, w.dt, H.PREC_FP64, w.lu_tol)
    u = dev(w.u0)
    H.step(f64, u, w.steps)
    e64 = np.linalg.norm(host(u) - ref) / nref
    fmx = H.factor(op, w.dt, H.PREC_MIXED, 1e-6)
    u = dev(w.u0)
    H.step(fmx, u, w.steps, refine={"sweeps": 2})
    emx = np.linalg.norm(host(u) - ref) / nref
    assert e64 <= 1e-10, e64
    assert emx <= 1e-8, emx
