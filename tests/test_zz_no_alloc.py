"""GPU test of hlevy_solve_noalloc (through the C ABI): the solve that takes
its work vectors from the library's static scratch array gives the result of
hlevy_solve with one right-hand side, bit for bit (same kernels, same
arithmetic), on two calls in a row, the second with a smaller problem, and
the device's free memory does not move across a call."""
import numpy as np
import pytest

from oracle.levy_oracle import Problem, generator_dense
import workloads as W

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


def case(H, n, prec, lu_tol):
    w = W.config2(n=n, steps=1)
    prob = H.make_problem(w.dim, w.n, w.lo, w.hi, w.s, lam=w.lam, C_=w.C, a=w.a, b=w.b, c=w.c, r0=w.r0)
    op = H.assemble(prob, H.make_hparams(aca_tol=1e-10, max_rank=16))
    fac = H.factor(op, w.dt, prec, lu_tol)
    G = generator_dense(Problem(dim=1, n=w.n, lo=w.lo, hi=w.hi, a=w.a, b=tuple(w.b), c=w.c, s=w.s,
                                lam=w.lam, C=w.C, r0=w.r0))
    M = np.eye(w.N) - 0.5 * w.dt * G
    return w, op, fac, M


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_solve_matches_solve(H, prec):
    p, tol = (H.PREC_FP64, 1e-12) if prec == "fp64" else (H.PREC_MIXED, 1e-6)
    rng = np.random.Generator(np.random.PCG64(77))
    runs = []
    for n in (2000, 700):                       # the second call takes a smaller problem
        w, op, fac, M = case(H, n, p, tol)
        xt = rng.standard_normal(w.N)
        b = dev(M @ xt)
        x_ref = torch.zeros(w.N, dtype=torch.float64, device="cuda")
        x_new = torch.full((w.N,), float("nan"), dtype=torch.float64, device="cuda")
        ref_st = H.solve(fac, b, x_ref, refine={"sweeps": 2, "tol": 1e-11}, stats=True)
        st = H.solve_noalloc(fac, b, x_new, refine={"sweeps": 2, "tol": 1e-11}, stats=True)
        torch.cuda.synchronize()
        assert torch.equal(x_new, x_ref), n
        assert st["steps_done"] == 1 and st["checks"] == 1
        assert st["last_rel_residual"] == ref_st["last_rel_residual"]
        err = np.linalg.norm(x_new.cpu().numpy() - xt) / np.linalg.norm(xt)
        assert err < 1e-9, (n, err)
        runs.append((fac, op, b, x_new.clone()))
    # the first problem again after the smaller one: the scratch keeps no
    # state between calls that the result depends on
    fac, op, b, x_first = runs[0]
    x_again = torch.zeros_like(x_first)
    H.solve_noalloc(fac, b, x_again, refine={"sweeps": 2})
    torch.cuda.synchronize()
    x_plain = torch.zeros_like(x_first)
    H.solve(fac, b, x_plain, refine={"sweeps": 2})
    torch.cuda.synchronize()
    assert torch.equal(x_again, x_plain)


def test_noalloc_solve_allocates_nothing(H):
    w, op, fac, M = case(H, 1500, H.PREC_MIXED, 1e-6)
    b = dev(M @ np.ones(w.N))
    x = torch.zeros(w.N, dtype=torch.float64, device="cuda")
    H.solve_noalloc(fac, b, x, refine={"sweeps": 1, "tol": 1e-9}, stats=True)   # warm-up
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for _ in range(3):
        H.solve_noalloc(fac, b, x, refine={"sweeps": 1, "tol": 1e-9}, stats=True)
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0
    assert np.allclose(x.cpu().numpy(), 1.0, rtol=0, atol=1e-9)


def test_noalloc_solve_rejects_bad_arguments(H):
    w, op, fac, M = case(H, 700, H.PREC_MIXED, 1e-6)
    b = dev(np.ones(w.N))
    with pytest.raises(H.HlevyError):
        H.solve_noalloc(fac, b, b)                      # b and x alias
    with pytest.raises(H.HlevyError):
        H.solve_noalloc(fac, b, torch.zeros_like(b), refine={"sweeps": 65})
