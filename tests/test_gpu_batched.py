"""GPU parity of the batched worklist (hlevy_factor_batched +
hlevy_step_batched) through the C ABI.

Each problem of a batch must give what the single-problem path gives and
what the dense CPU oracle gives on the same seeded inputs.  The batched
factorisation runs the same per-problem arithmetic as the single one; only
the LDS strides of merged launches may differ, which does not change a
result beyond rounding, so batched and single results are compared at
1e-12 relative (not bit for bit).  Against the oracle the bars are those of
the single path: 1e-10 (FP64) and 1e-8 (mixed precision).
"""
import numpy as np
import pytest

from oracle.levy_oracle import Problem, cn_run, generator_dense
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


def assemble(H, w):
    p = H.make_problem(w.dim, w.n, w.lo, w.hi, w.s, lam=w.lam, C_=w.C, a=w.a, b=w.b, c=w.c, r0=w.r0)
    hp = H.make_hparams(leaf=w.leaf, eta=w.eta, n_block=w.n_block, aca_tol=w.aca_tol, max_rank=16)
    return H.assemble(p, hp)


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def small_batch(steps=20):
    """Problems of the batched workload's distribution at oracle-friendly
    sizes, plus the smallest trees: two leaves (N = 128, the minimum of
    twice the leaf size), a ragged split (N = 129) and N = 200."""
    ws = W.config4_instances(count=6, seed=8324, nmin_log2=9.0, nmax_log2=11.6, steps=steps)
    extra = W.config4_instances(count=3, seed=8325, nmin_log2=6.0, nmax_log2=7.0, steps=steps)
    for w, n in zip(extra, (128, 129, 200)):
        w.n = n
        w.u0 = W.bump_1d(W.grid_points(1, n, -1.0, 1.0), 0.1)
    return ws + extra


CASES = {"fp64": (0, 1e-12, 1e-10, None), "mixed": (1, 1e-6, 1e-8, {"sweeps": 1})}


@pytest.mark.parametrize("case", list(CASES))
def test_batched_matches_single_and_oracle(H, case):
    prec, lu_tol, bar, refine = CASES[case]
    ws = small_batch()
    ops = [assemble(H, w) for w in ws]
    facs = H.factor_batched(ops, [w.dt for w in ws], prec, lu_tol)
    us = [dev(w.u0) for w in ws]
    H.step_batched(facs, us, ws[0].steps, refine=refine)
    for w, op, u in zip(ws, ops, us):
        single = H.factor(op, w.dt, prec, lu_tol)
        v = dev(w.u0)
        H.step(single, v, w.steps, refine=refine)
        got, one = host(u), host(v)
        ref = cn_run(generator_dense(oracle_problem(w)), w.dt, w.steps, w.u0).u
        assert rel(got, one) <= 1e-12, (w.name, w.n, rel(got, one))
        assert rel(got, ref) <= bar, (w.name, w.n, rel(got, ref))


def test_batched_groups_and_single_member(H):
    """A workspace budget that forces one problem per group, and a batch of
    one problem, give the results of the one-group batch."""
    ws = small_batch(steps=10)[:4]
    ops = [assemble(H, w) for w in ws]
    dts = [w.dt for w in ws]
    ref = H.factor_batched(ops, dts, 1, 1e-6)
    grp = H.factor_batched(ops, dts, 1, 1e-6, workspace_bytes=1)
    ua = [dev(w.u0) for w in ws]
    ub = [dev(w.u0) for w in ws]
    H.step_batched(ref, ua, 10, refine={"sweeps": 1})
    H.step_batched(grp, ub, 10, refine={"sweeps": 1})
    for a, b in zip(ua, ub):
        assert rel(host(b), host(a)) <= 1e-12
    one = H.factor_batched(ops[:1], dts[:1], 1, 1e-6)
    uc = dev(ws[0].u0)
    H.step_batched(one, [uc], 10, refine={"sweeps": 1})
    assert rel(host(uc), host(ua[0])) <= 1e-12
    # zero steps leave u untouched, zero sweeps take the preconditioner alone
    ud = dev(ws[1].u0)
    H.step_batched(one + [ref[1]], [dev(ws[0].u0), ud], 0)
    assert np.array_equal(host(ud), ws[1].u0)
    ue, uf = dev(ws[2].u0), dev(ws[2].u0)
    H.step_batched([ref[2]], [ue], 5, refine={"sweeps": 0})
    H.step(ref[2], uf, 5, refine={"sweeps": 0})
    assert rel(host(ue), host(uf)) <= 1e-12


def test_batched_rejects_bad_arguments(H):
    ws = small_batch(steps=1)[:2]
    ops = [assemble(H, w) for w in ws]
    facs = H.factor_batched(ops, [w.dt for w in ws], 1, 1e-6)
    u = dev(ws[0].u0)
    with pytest.raises(H.HlevyError, match="twice"):
        H.step_batched([facs[0], facs[0]], [u, dev(ws[0].u0)], 1)
    with pytest.raises(H.HlevyError, match="dt"):
        H.factor_batched(ops, [1e-3, -1.0], 1, 1e-6)
    with pytest.raises(H.HlevyError, match="lu_tol"):
        H.factor_batched(ops, [1e-3, 1e-3], 1, 2.0)


@pytest.fixture(scope="module")
def full_batch(H):
    """The batched workload at its full size: 512 problems, N log-uniform in
    [2^10, 2^15], mixed precision, 100 steps of dt = 1e-3."""
    ws = W.config4_instances()
    ops = [assemble(H, w) for w in ws]
    facs = H.factor_batched(ops, [w.dt for w in ws], 1, 1e-6)
    us = [dev(w.u0) for w in ws]
    H.step_batched(facs, us, ws[0].steps, refine={"sweeps": 1})
    return ws, ops, us


def test_full_batch_sampled(H, full_batch):
    """Seeded sample of the 512 problems: four with N <= 4096 against the
    oracle (mixed bar 1e-8), four larger ones against the single path."""
    ws, ops, us = full_batch
    rng = np.random.Generator(np.random.PCG64(357))
    small = [i for i, w in enumerate(ws) if w.n <= 4096]
    large = [i for i, w in enumerate(ws) if w.n > 4096]
    for i in rng.choice(small, 4, replace=False):
        w = ws[i]
        ref = cn_run(generator_dense(oracle_problem(w)), w.dt, w.steps, w.u0).u
        assert rel(host(us[i]), ref) <= 1e-8, (i, w.n)
    for i in rng.choice(large, 4, replace=False):
        w = ws[i]
        f = H.factor(ops[i], w.dt, 1, 1e-6)
        v = dev(w.u0)
        H.step(f, v, w.steps, refine={"sweeps": 1})
        assert rel(host(us[i]), host(v)) <= 1e-12, (i, w.n)
    for u in us:
        assert torch.isfinite(u).all()


def test_full_batch_vs_stored_oracle(H, full_batch):
    """Every problem of the 512 with N <= 4096 and 32 seeded larger ones
    (N up to 32559) against the oracle's results stored by
    tests/golden/make_batched_goldens.py: u at the last step on 512 seeded
    positions, relative error on those positions <= 1e-8 (the mixed bar).
    Every operator of the batch is built without a rank overflow."""
    import json
    import os
    gdir = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    path = os.path.join(gdir, "batched512_sample.json")
    if not os.path.exists(path):
        pytest.skip("no stored oracle results for the batched workload")
    meta = json.load(open(path))
    gold = np.load(os.path.join(gdir, "batched512_sample.npz"))
    ws, ops, us = full_batch
    assert meta["problems"] == len(ws)
    for op in ops:
        assert H.op_info(op)["rank_overflows"] == 0
    checked, worst = 0, 0.0
    for key, ent in meta["entries"].items():
        i = int(key)
        assert ent["key"] == W.workload_key(ws[i])
        pos, ref = gold["p%d" % i], gold["u%d" % i]
        err = rel(host(us[i])[pos], ref)
        worst = max(worst, err)
        assert err <= 1e-8, (i, ws[i].n, err)
        checked += 1
    assert checked == len(meta["small"]) + len(meta["large"])
    print(f"batched vs oracle: {checked} problems, worst {worst:.2e}")


def test_batched_assembly_equals_single(H):
    """hlevy_assemble_batched gives, problem by problem, the operator
    hlevy_assemble gives (bit for bit: the same kernels per problem), also
    with two different ACA tolerances in one batch."""
    ws = small_batch(steps=1)[:5]
    ws[1] = ws[1].with_(aca_tol=1e-8)
    probs, hps = [], []
    for w in ws:
        probs.append(H.make_problem(w.dim, w.n, w.lo, w.hi, w.s, lam=w.lam, C_=w.C, a=w.a, b=w.b, c=w.c, r0=w.r0))
        hps.append(H.make_hparams(leaf=w.leaf, eta=w.eta, n_block=w.n_block, aca_tol=w.aca_tol, max_rank=16))
    ops = H.assemble_batched(probs, hps)
    for w, p, hp, ob in zip(ws, probs, hps, ops):
        os_ = H.assemble(p, hp)
        da = torch.empty(w.N * w.N, dtype=torch.float64, device="cuda")
        db = torch.empty_like(da)
        H.op_densify(ob, da)
        H.op_densify(os_, db)
        assert torch.equal(da, db), w.name
