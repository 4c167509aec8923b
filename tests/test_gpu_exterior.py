"""GPU tests of the forcing of a non-zero exterior (hlevy_exterior_forcing,
1D) through the C ABI: against the oracle's exterior forcing for a symmetric
and an asymmetric measure, the constant identity G 1 + g(1) = -T, and a
Crank-Nicolson run whose exterior holds a fixed profile (g with phi = 1)
against the oracle's CN with the same forcing (FP64 1e-10, mixed 1e-8).
"""
import numpy as np
import pytest

from oracle.levy_oracle import Problem, cn_run, exterior_forcing, far_field, generator_dense, quadrature_constants

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1812_08324_amd import hlevy
    return hlevy


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


CASES = {
    "tempered_n1000": Problem(dim=1, n=1000, lo=-1.0, hi=1.0, s=0.75, lam=1.0, C=0.3, a=0.05, b=(0.5, 0.0)),
    "asym_n777": Problem(dim=1, n=777, lo=-1.0, hi=1.0, s=0.6, lam=0.5, lam_neg=3.0, C=0.4, a=0.02,
                         b=(0.3, 0.0)),
}


def assemble(H, p):
    prob = H.make_problem(1, p.n, p.lo, p.hi, p.s, lam=p.lam, C_=p.C, a=p.a, b=p.b, c=p.c, r0=p.r0,
                          lam_neg=p.lam_neg)
    return H.assemble(prob, H.make_hparams(aca_tol=1e-10, max_rank=16))


def exterior_profile(p):
    """A payoff-like exterior: 1 - e^{x} on the left (x < lo), e^{-x} - 1 on
    the right, on the 2 (n + 1) lattice points."""
    h = (p.hi - p.lo) / (p.n + 1)
    NW = p.n + 1
    left = p.lo + h * np.arange(-NW + 1, 1)
    right = p.hi + h * np.arange(0, NW)
    return np.concatenate([1.0 - np.exp(left), np.exp(-right) - 1.0])


@pytest.mark.parametrize("name", list(CASES))
def test_exterior_forcing_matches_oracle(H, name):
    p = CASES[name]
    op = assemble(H, p)
    ue = exterior_profile(p)
    g = torch.empty(p.n, dtype=torch.float64, device="cuda")
    H.exterior_forcing(op, dev(ue), g)
    ref = exterior_forcing(p, ue)
    assert rel(host(g), ref) <= 1e-13
    # a constant inside and out: G 1 + g(1) = -T in every row
    one = torch.ones(p.n, dtype=torch.float64, device="cuda")
    g1 = torch.empty_like(g)
    H.exterior_forcing(op, dev(np.ones(2 * (p.n + 1))), g1)
    y = torch.empty_like(g)
    H.matvec(op, one, y)
    T = quadrature_constants(p)["T"]
    scale = float(np.abs(host(g1)).max())
    assert np.abs(host(y) + host(g1) + T).max() <= 1e-9 * scale


def test_cn_with_exterior_forcing(H):
    """The exterior held at the profile above: each step's forcing is
    dt/2 (g + g) with phi = 1 (eq. equ:scheme with a constant source)."""
    p = CASES["asym_n777"]
    op = assemble(H, p)
    ue = exterior_profile(p)
    g = torch.empty(p.n, dtype=torch.float64, device="cuda")
    H.exterior_forcing(op, dev(ue), g)
    x = np.linspace(p.lo, p.hi, p.n + 2)[1:-1]
    u0 = np.exp(-x ** 2 / 0.02)
    dt, steps = 1e-3, 40
    phi = np.ones(steps + 1)
    ref = cn_run(generator_dense(p), dt, steps, u0, host(g), phi).u
    for prec, lu_tol, bar in ((H.PREC_FP64, 1e-12, 1e-10), (H.PREC_MIXED, 1e-6, 1e-8)):
        f = H.factor(op, dt, prec, lu_tol)
        u = dev(u0)
        H.step(f, u, steps, g=g, phi=phi, refine={"sweeps": 1})
        assert rel(host(u), ref) <= bar, prec


def test_exterior_forcing_rejects(H):
    """Overlapping u_ext and g, and a masked 2D operator, are refused before
    any device work."""
    op = assemble(H, CASES["tempered_n1000"])
    buf = torch.zeros(2 * 1001 + 1000, dtype=torch.float64, device="cuda")
    assert H.lib.hlevy_exterior_forcing(op.h, buf.data_ptr(), buf.data_ptr() + 8 * 10, None) == -1
    from workloads import lshape_mask
    op2 = H.assemble(H.make_problem(2, 24, -1.0, 1.0, 0.5, mask=lshape_mask(24)),
                     H.make_hparams(leaf=32, aca_tol=1e-8, max_rank=32))
    big = torch.zeros(74 * 74, dtype=torch.float64, device="cuda")
    out = torch.zeros(op2.N, dtype=torch.float64, device="cuda")
    assert H.lib.hlevy_exterior_forcing(op2.h, big.data_ptr(), out.data_ptr(), None) == -1


EXT2 = {
    "tempered2d_n20": Problem(dim=2, n=20, lo=-1.0, hi=1.0, s=0.6, lam=0.8, C=0.4, a=0.02, b=(0.3, -0.2)),
    "tilted2d_n17": Problem(dim=2, n=17, lo=-1.0, hi=1.0, s=0.5, lam=0.5, lam_neg=2.5, C=0.4, a=0.02,
                            b=(0.1, 0.2)),
}


@pytest.mark.parametrize("name", list(EXT2))
def test_exterior_forcing_2d(H, name):
    """2D exterior forcing on the extended lattice against the oracle (a
    smooth payoff-like exterior), and the constant identity G 1 + g(1) = -T
    through the H-matrix."""
    p = EXT2[name]
    prob = H.make_problem(2, p.n, p.lo, p.hi, p.s, lam=p.lam, C_=p.C, a=p.a, b=p.b, c=p.c, r0=p.r0,
                          lam_neg=p.lam_neg)
    op = H.assemble(prob, H.make_hparams(aca_tol=1e-8, max_rank=32))
    n, NW = p.n, p.n + 1
    h = (p.hi - p.lo) / (n + 1)
    idx = np.arange(-NW, n + NW)
    A1, A2 = np.meshgrid(p.lo + (idx + 1) * h, p.lo + (idx + 1) * h, indexing="ij")
    ue = (np.exp(-0.5 * (A1 ** 2 + A2 ** 2)) * np.cos(A1 - 0.3 * A2)).ravel()
    g = torch.empty(p.N, dtype=torch.float64, device="cuda")
    H.exterior_forcing(op, dev(ue), g)
    ref = exterior_forcing(p, ue)
    assert rel(host(g), ref) <= 1e-13
    H.exterior_forcing(op, dev(np.ones_like(ue)), g)
    y = torch.empty_like(g)
    H.matvec(op, dev(np.ones(p.N)), y)
    T = quadrature_constants(p)["T"]
    scale = float(np.abs(host(g)).max())
    assert np.abs(host(y) + host(g) + T).max() <= 1e-7 * scale


FAR = {
    "tempered_n400": Problem(dim=1, n=400, lo=-1.0, hi=1.0, s=0.75, lam=1.0, C=0.3, a=0.05, b=(0.5, 0.0)),
    "asym_n377": Problem(dim=1, n=377, lo=-1.0, hi=1.0, s=0.6, lam=0.5, lam_neg=3.0, C=0.4, a=0.02, b=(0.3, 0.0)),
}


def extended_profile(p, nxt):
    """The payoff-like exterior on next lattice points per side."""
    h = (p.hi - p.lo) / (p.n + 1)
    left = p.lo + h * np.arange(-nxt + 1, 1)
    right = p.hi + h * np.arange(0, nxt)
    return np.concatenate([1.0 - np.exp(left), np.exp(-right) - 1.0])


@pytest.mark.parametrize("name", list(FAR))
def test_far_field_matches_oracle(H, name):
    """hlevy_exterior_forcing_far against the oracle's window forcing plus
    far field (extended lattice of 2 (n + 1) + 5 points per side, tails 1 on
    the left and -1 on the right: the profile's limits)."""
    p = FAR[name]
    op = assemble(H, p)
    nxt = 2 * (p.n + 1) + 5
    ue = extended_profile(p, nxt)
    g = torch.empty(p.n, dtype=torch.float64, device="cuda")
    H.exterior_forcing_far(op, dev(ue), nxt, 1.0, -1.0, g)
    NW = p.n + 1
    ref = exterior_forcing(p, ue[nxt - NW: nxt + NW]) + far_field(p, ue, nxt, 1.0, -1.0)
    assert rel(host(g), ref) <= 1e-13


def test_far_field_edges_and_constant(H):
    """next = n + 1 with zero tails is hlevy_exterior_forcing bit for bit; a
    constant exterior with the same constant tails completes G c + g + f = 0;
    next below n + 1 and non-finite tails are refused."""
    p = FAR["asym_n377"]
    op = assemble(H, p)
    NW = p.n + 1
    ue = dev(exterior_profile(p))
    a = torch.empty(p.n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    H.exterior_forcing(op, ue, a)
    H.exterior_forcing_far(op, ue, NW, 0.0, 0.0, b)
    assert torch.equal(a, b)
    c = 0.7
    H.exterior_forcing_far(op, dev(np.full(2 * NW, c)), NW, c, c, b)
    y = torch.empty_like(a)
    H.matvec(op, dev(np.full(p.n, c)), y)
    scale = float(np.abs(host(b)).max())
    assert np.abs(host(y) + host(b)).max() <= 1e-9 * scale
    with pytest.raises(H.HlevyError, match="next"):
        H.exterior_forcing_far(op, dev(np.zeros(2 * p.n)), p.n, 0.0, 0.0, b)
    with pytest.raises(H.HlevyError, match="tail"):
        H.exterior_forcing_far(op, ue, NW, float("nan"), 0.0, b)



def _assemble2(H, p):
    prob = H.make_problem(2, p.n, p.lo, p.hi, p.s, lam=p.lam, C_=p.C, a=p.a, b=p.b, c=p.c, r0=p.r0,
                          lam_neg=p.lam_neg)
    return H.assemble(prob, H.make_hparams(aca_tol=1e-8, max_rank=32))


def _extended2(p, nxt):
    """A smooth exterior on the 2D lattice of indices -nxt .. n - 1 + nxt."""
    h = (p.hi - p.lo) / (p.n + 1)
    idx = np.arange(-nxt, p.n + nxt)
    A1, A2 = np.meshgrid(p.lo + (idx + 1) * h, p.lo + (idx + 1) * h, indexing="ij")
    return (np.exp(-0.3 * (A1 ** 2 + A2 ** 2)) * np.cos(A1 - 0.3 * A2)).ravel()


@pytest.mark.parametrize("name", list(EXT2))
def test_far_field_2d_matches_oracle(H, name):
    """2D hlevy_exterior_forcing_far against the oracle's window forcing plus
    far field: an extended lattice reaching 9 points past the window, tails
    0.3 (y1 < 0) and -0.2 (y1 > 0).  FP64 on both sides; the GPU takes the
    half-plane tails by a 32-node Gauss-Legendre rule per octant of an
    analytic integrand, the oracle by adaptive quadrature."""
    p = EXT2[name]
    op = _assemble2(H, p)
    n, NW = p.n, p.n + 1
    nxt = NW + 9
    ue = _extended2(p, nxt)
    g = torch.empty(p.N, dtype=torch.float64, device="cuda")
    H.exterior_forcing_far(op, dev(ue), nxt, 0.3, -0.2, g)
    side = n + 2 * nxt
    o = nxt - NW
    win = ue.reshape(side, side)[o:o + 3 * n + 2, o:o + 3 * n + 2].ravel()
    ref = exterior_forcing(p, win) + far_field(p, ue, nxt, 0.3, -0.2)
    assert rel(host(g), ref) <= 1e-12


def test_far_field_2d_edges_and_constant(H):
    """2D: next = n + 1 with zero tails is hlevy_exterior_forcing bit for
    bit; a constant exterior with the same constant tails completes
    G c + g + f = 0 through the H-matrix; next below n + 1 is refused."""
    p = EXT2["tilted2d_n17"]
    op = _assemble2(H, p)
    n, NW = p.n, p.n + 1
    ue = dev(_extended2(p, NW))
    a = torch.empty(p.N, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    H.exterior_forcing(op, ue, a)
    H.exterior_forcing_far(op, ue, NW, 0.0, 0.0, b)
    assert torch.equal(a, b)
    c = 0.7
    H.exterior_forcing_far(op, dev(np.full((3 * n + 2) ** 2, c)), NW, c, c, b)
    y = torch.empty_like(a)
    H.matvec(op, dev(np.full(p.N, c)), y)
    scale = float(np.abs(host(b)).max())
    assert np.abs(host(y) + host(b)).max() <= 1e-7 * scale
    with pytest.raises(H.HlevyError, match="next"):
        H.exterior_forcing_far(op, dev(np.zeros((3 * n) ** 2)), n, 0.0, 0.0, b)


@pytest.mark.parametrize("dim,lam_neg", [(1, None), (1, 2.0), (2, None), (2, 2.5)])
def test_tempered_half_index_tail(H, dim, lam_neg):
    """s = 1/2 with tempering: the measure beyond the window needs
    Gamma(-1, x), which the recursion of the incomplete gamma function takes
    through Gamma(0, x) = E1(x); the constants against the oracle's
    quadrature."""
    n = 300 if dim == 1 else 20
    p = Problem(dim=dim, n=n, lo=-1.0, hi=1.0, s=0.5, lam=0.7, lam_neg=lam_neg, C=0.4)
    prob = H.make_problem(dim, n, p.lo, p.hi, 0.5, lam=0.7, C_=0.4, lam_neg=lam_neg)
    op = H.assemble(prob, H.make_hparams(aca_tol=1e-8, max_rank=32))
    ref = quadrature_constants(p)
    for v, key in zip(H.op_constants(op), ("S0", "S2", "C2", "T")):
        assert v == pytest.approx(ref[key], rel=1e-11), key
