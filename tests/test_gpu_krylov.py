"""GPU tests of the steady solves (hlevy_krylov_solve) through the C ABI.

(shift I - G) x = b by conjugate gradients or BiCGSTAB with the factor's
inverse factors as the preconditioner (Sec. 5.1, 5.3, 5.4), against the
oracle's dense solve of the same system (plain definition: dense LU) and,
for the fractional Poisson problem, against its closed form (Sec. 5.3).
The GPU solves the H-matrix system, the oracle the dense one: the bar
covers the H-matrix error of the operator (ACA at 1e-10 or 1e-8) on top of
the iteration's tolerance (1e-12).
"""
import numpy as np
import pytest

from oracle.levy_oracle import (Problem, fractional_poisson_exact, generator_dense, grid, steady_residual,
                                steady_solve)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_08324_amd import hlevy
    return hlevy


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def build(H, p, aca_tol=1e-10, max_rank=16, dt=1e4, prec=1, lu_tol=1e-6):
    hp = H.make_problem(p.dim, p.n, p.lo, p.hi, p.s, lam=p.lam, C_=p.C, a=p.a, b=p.b, c=p.c, r0=p.r0)
    op = H.assemble(hp, H.make_hparams(aca_tol=aca_tol, max_rank=max_rank))
    return op, H.factor(op, dt, prec, lu_tol)


POISSON = {
    "frac1d_s0.25_n1023": (Problem(dim=1, n=1023, lo=-1.0, hi=1.0, s=0.25), 1e-10),
    "frac1d_s0.5_n1023": (Problem(dim=1, n=1023, lo=-1.0, hi=1.0, s=0.5), 1e-10),
    "frac1d_s0.75_n2000": (Problem(dim=1, n=2000, lo=-1.0, hi=1.0, s=0.75), 1e-10),
    "frac2d_s0.5_33x33": (Problem(dim=2, n=33, lo=0.0, hi=1.0, s=0.5), 1e-10),
}


@pytest.mark.parametrize("name", list(POISSON))
def test_fractional_poisson_cg(H, name):
    """(-Delta)^s u = 1 with zero exterior (shift 0, fractional generator),
    conjugate gradients preconditioned by the mixed factor of
    I + dt/2 (-G) with dt = 1e4: converged to 1e-12 within 12 iterations,
    equal to the oracle's dense solve, and in 1D as close to the closed form
    as the oracle is.  Without the preconditioner the same tolerance takes
    at least ten times more iterations."""
    p, bar = POISSON[name]
    aca = 1e-10 if p.dim == 1 else 1e-8
    op, fac = build(H, p, aca_tol=aca, max_rank=16 if p.dim == 1 else 32)
    f = np.ones(p.N)
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    st = H.krylov_solve(fac, dev(f), x, method=H.KRYLOV_CG, max_iter=200, tol=1e-12)
    assert st["converged"] and st["iterations"] <= 12, st
    assert st["rel_residual"] <= 1e-11, st
    G = generator_dense(p)
    ref = steady_solve(G, 0.0, f)
    got = host(x)
    err = rel(got, ref)
    print(f"{name}: {st['iterations']} iterations, rel residual {st['rel_residual']:.2e}, vs oracle {err:.2e}")
    assert err <= bar, err
    assert steady_residual(G, 0.0, got, f) <= 1e3 * bar
    if p.dim == 1:
        ex = fractional_poisson_exact(1, p.s, grid(p))
        assert abs(rel(got, ex) - rel(ref, ex)) <= 1e-8
    hist = st["history"]
    assert len(hist) == st["iterations"] + 1 and hist[0] == pytest.approx(1.0) and hist[-1] <= 1e-12
    plain = torch.zeros_like(x)
    s0 = H.krylov_solve(fac, dev(f), plain, method=H.KRYLOV_CG, max_iter=20 * st["iterations"] + 20, tol=1e-12,
                        precondition=False, raise_not_converged=False)
    assert s0["iterations"] >= 10 * st["iterations"], (s0["iterations"], st["iterations"])


def test_bicgstab_nonsymmetric_and_shifted(H):
    """The tempered operator with drift and diffusion (nonsymmetric) at
    N = 2000, shift = 2/dt: the steady system of the Crank-Nicolson matrix
    scaled by 2/dt.  BiCGSTAB with the mixed factor of the same dt meets
    1e-12 in a few iterations and equals the oracle's dense solve.  The
    symmetric fractional case gives CG's solution."""
    dt = 1e-3
    p = Problem(dim=1, n=2000, lo=-1.0, hi=1.0, s=0.75, lam=1.0, a=0.05, b=(0.5, 0.0),
                C=None)
    op, fac = build(H, p, dt=dt)
    x0 = grid(p)[:, 0]
    f = np.exp(-x0 ** 2 / 0.02) + 0.1 * np.sin(3 * x0)
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    st = H.krylov_solve(fac, dev(f), x, method=H.KRYLOV_BICGSTAB, max_iter=50, tol=1e-12, shift=2.0 / dt)
    assert st["converged"] and st["iterations"] <= 5, st
    ref = steady_solve(generator_dense(p), 2.0 / dt, f)
    err = rel(host(x), ref)
    print(f"BiCGSTAB tempered: {st['iterations']} iterations, vs oracle {err:.2e}")
    assert err <= 1e-10, err
    q = Problem(dim=1, n=1023, lo=-1.0, hi=1.0, s=0.5)
    op2, fac2 = build(H, q)
    a = torch.zeros(q.N, dtype=torch.float64, device="cuda")
    b = torch.zeros_like(a)
    H.krylov_solve(fac2, dev(np.ones(q.N)), a, method=H.KRYLOV_CG, tol=1e-13)
    H.krylov_solve(fac2, dev(np.ones(q.N)), b, method=H.KRYLOV_BICGSTAB, tol=1e-13)
    assert rel(host(b), host(a)) <= 1e-11


def test_krylov_edges(H):
    """Zero right-hand side: x = 0 after no iteration.  A converged guess:
    no iteration.  max_iter 1 at an unreachable tolerance: NOT_CONVERGED
    with the last iterate in x (finite, better than x = 0).  FP64 factor as
    the preconditioner.  Bad options: INVALID_ARG."""
    p = Problem(dim=1, n=700, lo=-1.0, hi=1.0, s=0.5)
    op, fac = build(H, p)
    f = dev(np.ones(p.N))
    x = dev(np.full(p.N, 5.0))
    st = H.krylov_solve(fac, torch.zeros_like(f), x)
    assert st["iterations"] == 0 and st["converged"] and not torch.any(x != 0)
    H.krylov_solve(fac, f, x, tol=1e-13)
    st = H.krylov_solve(fac, f, x, tol=1e-11, use_guess=True)
    assert st["iterations"] == 0 and st["converged"]
    y = torch.zeros_like(x)
    with pytest.raises(H.HlevyError, match="NOT_CONVERGED"):
        H.krylov_solve(fac, f, y, max_iter=1, tol=1e-15)
    got = host(y)
    assert np.isfinite(got).all() and rel(got, host(x)) < 1.0
    f64 = H.factor(op, 1e4, H.PREC_FP64, 1e-12)
    z = torch.zeros_like(x)
    st = H.krylov_solve(f64, f, z, tol=1e-13)
    assert st["converged"] and st["iterations"] <= 6 and rel(host(z), host(x)) <= 1e-12
    for kw, msg in (({"method": 7}, "method"), ({"max_iter": 0}, "max_iter"), ({"tol": -1.0}, "tol"),
                    ({"shift": float("nan")}, "shift")):
        with pytest.raises(H.HlevyError, match=msg):
            H.krylov_solve(fac, f, z, **kw)
    with pytest.raises(H.HlevyError, match="overlap"):
        H.krylov_solve(fac, f, f)


def test_gmres_matches_bicgstab_and_oracle(H):
    """Restarted right-preconditioned GMRES on the nonsymmetric tempered
    operator (drift and diffusion, N = 2000, shift 2/dt): converges to 1e-12
    in a few steps and equals the oracle's dense solve; its history (the
    Givens estimate) decreases monotonically; GMRES(1) (a restart after
    every step) still converges to the same solution; without the preconditioner it needs
    far more steps; restart out of range is refused."""
    dt = 1e-3
    p = Problem(dim=1, n=2000, lo=-1.0, hi=1.0, s=0.75, lam=1.0, a=0.05, b=(0.5, 0.0), C=None)
    op, fac = build(H, p, dt=dt)
    x0 = grid(p)[:, 0]
    f = np.exp(-x0 ** 2 / 0.02) + 0.1 * np.sin(3 * x0)
    ref = steady_solve(generator_dense(p), 2.0 / dt, f)
    x = torch.zeros(p.N, dtype=torch.float64, device="cuda")
    st = H.krylov_solve(fac, dev(f), x, method=H.KRYLOV_GMRES, max_iter=50, tol=1e-12, shift=2.0 / dt)
    assert st["converged"] and st["iterations"] <= 6 and st["rel_residual"] <= 1e-11, st
    assert rel(host(x), ref) <= 1e-10
    hist = st["history"]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))
    y = torch.zeros_like(x)
    s2 = H.krylov_solve(fac, dev(f), y, method=H.KRYLOV_GMRES, max_iter=60, tol=1e-12, shift=2.0 / dt, restart=1)
    assert s2["converged"] and rel(host(y), ref) <= 1e-10, s2
    z = torch.zeros_like(x)
    s0 = H.krylov_solve(fac, dev(f), z, method=H.KRYLOV_GMRES, max_iter=600, tol=1e-12, shift=2.0 / dt,
                        precondition=False, restart=20, raise_not_converged=False)
    assert s0["iterations"] >= 5 * st["iterations"], (s0["iterations"], st["iterations"])
    if s0["converged"]:       # across restarts of 20 steps
        assert rel(host(z), ref) <= 1e-9
    with pytest.raises(H.HlevyError, match="restart"):
        H.krylov_solve(fac, dev(f), z, method=H.KRYLOV_GMRES, restart=65)
    print(f"GMRES: {st['iterations']} steps (restart 1: {s2['iterations']}), without preconditioner "
          f"{s0['iterations']} (converged {s0['converged']})")


def test_gmres_variable_order_lshape(H):
    """GMRES on the variable-order L-shaped problem (Sec. 5.4), the eps1
    factor preconditioning the accurate operator: the oracle's dense solve."""
    from oracle.levy_oracle import variable_order_generator
    from workloads import variable_order_lshape
    w = variable_order_lshape(30)
    prob = H.make_problem(2, 30, -1.0, 1.0, 0.5, mask=w["mask"], s_field=w["s"])
    fine = H.assemble(prob, H.make_hparams(leaf=32, aca_tol=1e-10, cluster=H.CLUSTER_KMEANS))
    coarse = H.assemble(prob, H.make_hparams(leaf=32, aca_tol=1e-4, cluster=H.CLUSTER_KMEANS))
    fac = H.factor(coarse, 1e8, H.PREC_FP64, 1e-10)
    u = torch.zeros(w["N"], dtype=torch.float64, device="cuda")
    st = H.krylov_solve(fac, dev(-w["f"]), u, method=H.KRYLOV_GMRES, max_iter=50, tol=1e-12, op=fine)
    assert st["converged"] and st["iterations"] <= 5, st
    G = variable_order_generator(Problem(dim=2, n=30, lo=-1.0, hi=1.0, s=0.5), w["mask"], w["s"])
    assert rel(host(u), steady_solve(G, 0.0, -w["f"])) <= 1e-9
