"""Plain CPU FP64 oracle for the Crank-Nicolson / Levy-generator path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The product path
(the HIP library and its Python binding) never imports, calls or links it, and
this module imports nothing from the product package.

What it computes (Xu & Darve, arXiv 1812.08324):

* the discrete generator ``G`` of the model equation (Sec. 3.1, eq. equ:ut):
  diffusion ``a*Laplacian_h``, drift ``b*D_h`` (central difference), killing
  ``c``, and the jump operator discretised by singularity subtraction
  (Sec. 4, eqs. equ:evalIx1d, equ:I1approx, equ:I2approx, equ:I3approx),
  as a plain dense matrix, one row at a time;
* the Crank-Nicolson recursion (Sec. 3.2, eq. equ:scheme) with the
  trapezoidal forcing term, solved by dense LU with partial pivoting
  (LAPACK getrf/getrs through scipy);
* the steady problems (shift I - G) u = f that the H-LU preconditions in an
  iteration (Sec. 5.1; the fractional Poisson problem of Sec. 5.3 is
  shift = 0 with the fractional generator), solved by the same dense LU;
* the forcing of a non-zero exterior (Sec. 4: the window terms that reach
  outside the box, 1D and 2D) and the far-field term f^{L_W} of
  equ:I2approx (eq. equ:fxy) on an extended lattice with constant tails;
* the fixed-rank Taylor factors of the Gaussian kernel's admissible blocks
  (Sec. 3.3, Lemma 1).

Nothing here is blocked, compressed or reordered: the H-matrix method must
reproduce these results up to its truncation tolerance.

Readings of the paper taken here (the paper is garbled or silent on them):

* Sign convention.  The paper writes ``A = -G``; here ``G`` is the generator,
  ``M = I - dt/2 G`` and ``Mp = I + dt/2 G`` (Sec. 3.2, eq. equ:Aij).
* Window ``rho``: the indicator of the infinity-norm ball of radius
  ``r = m*h`` with ``m = floor(r0/h + 1/2)``, weight 1/2 on its boundary nodes
  (Sec. 4, eq. equ:rho_condition leaves the shape open).  In 2D it is the
  product of the 1D node weights.
* The u'' term of equ:I1approx carries the trapezoid weights ``w_j``
  (dimensionally required); the u' term vanishes for the symmetric kernels
  used here.  Net local term: ``(C2 - S2)/2 * Laplacian_h u``.
* The window half-width ``L_W`` equals the domain extent, so every in-domain
  offset lies inside the window and the far field ``f^{L_W}`` is zero under
  the zero-exterior condition (Sec. 4, closing remark); a non-zero exterior
  enters through the exterior forcing and the far field below.
* In 2D the singularity subtraction uses ``int rho nu y_i y_j = delta_ij C2``
  (radial kernel, square window), giving the 5-point Laplacian.
* Asymmetric 1D measures (rate lam for y > 0, lam_neg for y < 0): the
  generator keeps the compensator of equ:I1approx, L u = int (u(x+y) - u(x)
  - rho(y) y u'(x)) nu(y) dy, so the u' sum of I1 is not added back; it is
  discretised with the trapezoid weights and the central difference
  (u_{i+1} - u_{i-1}) / (2h) (the printed /h without weights is
  dimensionally off).  Another compensator differs by a drift, which the
  caller can fold into b.
* Variable jump index (Sec. 5.4): the paper applies the discretisation of
  Sec. 4 to -(-Delta)^{s(x)} without writing it out.  Read here: the row of
  x_i is the constant-order row with s = s(x_i) and kernel constant
  c_{d,s(x_i)} (its own quadrature constants), and u = 0 on the grid points
  outside the L-shaped domain, so those columns drop out.
* 2D asymmetric measures: the symmetric kernel tilted along the first
  axis, C exp(-lam0 |y| + theta y1) / |y|^(2+2s) with lam0 = (lam +
  lam_neg)/2 and theta = (lam_neg - lam)/2, so that the rates along that
  axis are those of the 1D measure; the compensator is kept as in 1D and
  each axis takes its own u'' coefficient.
* The far field f^{L_W} (which the paper leaves to an input or a
  quadrature): the trapezoid rule on the extended lattice beyond the window
  and, past the lattice, a constant per side (1D) or per half-plane of the
  first axis (2D) times the measure of that region.
* The closed-form solution of the 1D fractional Poisson problem (Sec. 5.3):
  the paper prints the factor 2^{2s} Gamma(1+s) Gamma((1+2s)/2)/Gamma(1/2)
  in front of (1-x^2)^s.  That factor is (-Delta)^s of (1-x^2)^s (the ball
  constant), so the solution of (-Delta)^s u = 1 carries its reciprocal.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np
import scipy.integrate as integrate
import scipy.linalg as sla
import scipy.special as sp

__all__ = [
    "Problem", "frac_const", "ball_const", "gauss_const", "grid", "h_of",
    "quadrature_constants", "generator_row", "generator_dense", "cn_matrices",
    "cn_run", "kernel_nu", "steady_solve", "steady_residual", "fractional_poisson_exact",
    "taylor_terms", "taylor_factors", "kernel_nu_signed", "exterior_forcing", "variable_order_generator",
    "far_field", "kernel_nu_tilted",
]


# ---------------------------------------------------------------------------
# Closed-form constants
# ---------------------------------------------------------------------------
def frac_const(d: int, s: float) -> float:
    """c_{d,s} = 4^s Gamma(d/2+s) / (pi^{d/2} |Gamma(-s)|)  (Sec. 1, Sec. 4)."""
    return 4.0 ** s * sp.gamma(d / 2.0 + s) / (math.pi ** (d / 2.0) * abs(sp.gamma(-s)))


def ball_const(d: int, s: float) -> float:
    """(-Delta)^s (1-|x|^2)_+^s on the unit ball:
    2^{2s} Gamma(1+s) Gamma(d/2+s) / Gamma(d/2)  (Sec. 5.3, eq. equ:u1)."""
    return 4.0 ** s * sp.gamma(1.0 + s) * sp.gamma(d / 2.0 + s) / sp.gamma(d / 2.0)


def gauss_const(d: int, s: float) -> float:
    """(-Delta)^s exp(-|x|^2) at x = 0: 4^s Gamma(d/2+s)/Gamma(d/2)
    (Sec. 5.3, eq. equ:u0 for d = 1)."""
    return 4.0 ** s * sp.gamma(d / 2.0 + s) / sp.gamma(d / 2.0)


# ---------------------------------------------------------------------------
# Problem description
# ---------------------------------------------------------------------------
@dataclass
class Problem:
    """Model equation u_t = a Lap u + b.grad u + c u + L u on a box with zero
    exterior (Sec. 3.1 eq. equ:ut; Sec. 4 closing remark).

    Jump kernel (kernel = "tempered") nu(y) = C exp(-lam |y|) / |y|^{d+2s};
    C = None selects c_{d,s} (then lam = 0 is exactly the fractional
    Laplacian, Sec. 4).  kernel = "gaussian": the Gaussian (Merton) jump
    density nu(y) = C exp(-eps2 |y|^2) (Sec. 3.3), C = None selects 1; it is
    bounded, so the generator is the plain trapezoid rule of Sec. 3.2
    (eqs. equ:dl, equ:Aij) without singularity subtraction.
    """
    dim: int
    n: int                       # interior points per axis
    lo: float = -1.0
    hi: float = 1.0
    a: float = 0.0
    b: tuple = (0.0, 0.0)
    c: float = 0.0
    s: float = 0.5
    lam: float = 0.0
    C: float | None = None
    r0: float = 0.2              # window radius before snapping to the grid
    jumps: bool = True           # False drops the jump operator (nu = 0)
    kernel: str = "tempered"     # or "gaussian"
    eps2: float = 0.0            # Gaussian kernel: nu(y) = C exp(-eps2 |y|^2)
    lam_neg: float | None = None  # tempered kernel: rate of the jumps y_1 < 0 (None: lam, symmetric); 2D: tilted

    @property
    def N(self) -> int:
        return self.n if self.dim == 1 else self.n * self.n

    @property
    def Cval(self) -> float:
        if self.C is not None:
            return float(self.C)
        return 1.0 if self.kernel == "gaussian" else frac_const(self.dim, self.s)


def h_of(p: Problem) -> float:
    return (p.hi - p.lo) / (p.n + 1)


def grid(p: Problem) -> np.ndarray:
    """Interior grid points, lexicographic order (first coordinate slowest).
    Returns an (N, dim) array."""
    h = h_of(p)
    x1 = p.lo + h * np.arange(1, p.n + 1, dtype=np.float64)
    if p.dim == 1:
        return x1[:, None]
    X, Y = np.meshgrid(x1, x1, indexing="ij")
    return np.stack([X.ravel(), Y.ravel()], axis=1)


def kernel_nu_signed(p: Problem, y):
    """The 1D tempered kernel at the signed jump y != 0: rate lam for y > 0,
    lam_neg for y < 0 (an asymmetric, CGMY-type measure when they differ)."""
    y = np.asarray(y, dtype=np.float64)
    lneg = p.lam if p.lam_neg is None else p.lam_neg
    rate = np.where(y > 0, p.lam, lneg)
    return p.Cval * np.exp(-rate * np.abs(y)) / np.abs(y) ** (1.0 + 2.0 * p.s)


def kernel_nu_tilted(p: Problem, y1, y2):
    """The 2D asymmetric tempered kernel at the jump (y1, y2) != 0: the
    symmetric kernel tilted along the first axis,
    C exp(-lam0 |y| + theta y1) / |y|^{2+2s} with lam0 = (lam + lam_neg)/2 and
    theta = (lam_neg - lam)/2, so that the rate along the first axis is lam
    for y1 > 0 and lam_neg for y1 < 0, as the 1D asymmetric kernel."""
    y1 = np.asarray(y1, dtype=np.float64)
    y2 = np.asarray(y2, dtype=np.float64)
    lam0, th = 0.5 * (p.lam + p.lam_neg), 0.5 * (p.lam_neg - p.lam)
    r = np.hypot(y1, y2)
    return p.Cval * np.exp(-lam0 * r + th * y1) / r ** (2.0 + 2.0 * p.s)


def kernel_nu(p: Problem, r):
    """nu at distance r > 0."""
    r = np.asarray(r, dtype=np.float64)
    if p.kernel == "gaussian":
        return p.Cval * np.exp(-p.eps2 * r * r)
    return p.Cval * np.exp(-p.lam * r) / r ** (p.dim + 2.0 * p.s)


# ---------------------------------------------------------------------------
# Quadrature constants of the singularity subtraction (Sec. 4)
# ---------------------------------------------------------------------------
def _trap_w(k, NW, h):
    """Trapezoid weights on the window grid: h inside, h/2 at |k| = NW."""
    k = np.abs(k)
    return np.where(k == NW, 0.5 * h, h)


def _rho_w(k, m):
    """Grid window weights: 1 inside, 1/2 on the boundary |k| = m, 0 outside."""
    k = np.abs(k)
    return np.where(k < m, 1.0, np.where(k == m, 0.5, 0.0))


def _Rtheta(theta):
    return 1.0 / np.maximum(np.abs(np.cos(theta)), np.abs(np.sin(theta)))


def _quad_theta(f):
    """int_0^{2 pi} f(theta) d theta, split at the corners of the square."""
    tot = 0.0
    for q in range(8):
        val, _ = integrate.quad(f, q * math.pi / 4, (q + 1) * math.pi / 4,
                                epsabs=0.0, epsrel=1e-13, limit=200)
        tot += val
    return tot


def quadrature_constants(p: Problem) -> dict:
    """S0, S2 (grid sums, zero offset excluded), C2 = int rho nu y_1^2 and
    T = int_{outside window} nu  (Sec. 4, equ:I1approx..equ:I3approx).

    S0 = sum' W_k nu(kh)                   (coefficient of -u_i in I1)
    S2 = sum' W_k rho_k nu(kh) (k_1 h)^2    (coefficient of the u'' term in I1)
    C2 = int rho(y) nu(y) y_1^2 dy          (local diffusion term I3)
    T  = int_{|y|_inf > L_W} nu(y) dy       (I2 with zero far field)
    """
    h = h_of(p)
    NW = p.n + 1                     # L_W = (n+1) h = domain extent
    LW = NW * h
    m = int(math.floor(p.r0 / h + 0.5))   # nearest grid multiple, ties rounded up
    r = m * h
    C, s, lam, d = p.Cval, p.s, p.lam, p.dim
    if not p.jumps:
        return dict(S0=0.0, S2=0.0, C2=0.0, T=0.0, h=h, NW=NW, m=m, r=r, LW=LW)
    if p.kernel == "gaussian":
        # Sec. 3.2 (equ:dl): the coefficient of -u_i is h^d sum' nu(kh) over
        # the whole lattice (the exterior holds u = 0, but u_i leaves to
        # every offset); no singularity subtraction, no window terms.  Terms
        # below 1e-18 nu(0) are dropped.
        K = int(math.ceil(math.sqrt(41.5 / p.eps2) / h)) + 1
        k = np.arange(-K, K + 1)
        if d == 1:
            kk = k[k != 0]
            S0 = h * math.fsum(kernel_nu(p, np.abs(kk) * h))
        else:
            K1, K2 = np.meshgrid(k, k, indexing="ij")
            sel = (K1 != 0) | (K2 != 0)
            S0 = h * h * math.fsum(kernel_nu(p, np.hypot(K1[sel] * h, K2[sel] * h)))
        return dict(S0=S0, S2=0.0, C2=0.0, T=0.0, h=h, NW=NW, m=m, r=r, LW=LW)
    k = np.arange(-NW, NW + 1)
    nz = k != 0
    if d == 1 and p.lam_neg is not None:
        # asymmetric measure (NEXT-3 reading): every sum and integral takes
        # each side with its own rate; S1 = sum' W_k rho_k nu(kh) (kh) is the
        # coefficient of the u' term of equ:I1approx, zero for symmetric nu
        kk = k[nz]
        w = _trap_w(kk, NW, h)
        nu = kernel_nu_signed(p, kk * h)
        rw = _rho_w(kk, m)
        S0 = math.fsum(w * nu)
        S2 = math.fsum(w * rw * nu * (kk * h) ** 2)
        S1 = math.fsum(w * rw * nu * (kk * h))
        a2 = 2.0 - 2.0 * s
        C2 = T = 0.0
        for rate in (lam, p.lam_neg):
            if rate == 0.0:
                C2 += C * r ** a2 / a2
                T += C * LW ** (-2.0 * s) / (2.0 * s)
            else:
                C2 += C * rate ** (-a2) * sp.gammainc(a2, rate * r) * sp.gamma(a2)
                val, _ = integrate.quad(lambda y: np.exp(-rate * y) * y ** (-1.0 - 2.0 * s),
                                        LW, np.inf, epsabs=0.0, epsrel=1e-13, limit=400)
                T += C * val
        return dict(S0=S0, S2=S2, C2=C2, T=T, S1=S1, h=h, NW=NW, m=m, r=r, LW=LW)
    if d == 2 and p.lam_neg is not None:
        # 2D asymmetric (tilted) measure: the u' sum S1 (first axis; the
        # second vanishes by the y2 -> -y2 symmetry) and the u'' sums and
        # integrals per axis (S2, C2 first axis, S2y, C2y second); the mixed
        # ones vanish by the same symmetry
        K1, K2 = np.meshgrid(k, k, indexing="ij")
        K1 = K1.ravel(); K2 = K2.ravel()
        nz2 = (K1 != 0) | (K2 != 0)
        K1 = K1[nz2]; K2 = K2[nz2]
        W = _trap_w(K1, NW, h) * _trap_w(K2, NW, h)
        nu = kernel_nu_tilted(p, K1 * h, K2 * h)
        rw = _rho_w(K1, m) * _rho_w(K2, m)
        S0 = math.fsum(W * nu)
        S2 = math.fsum(W * rw * nu * (K1 * h) ** 2)
        S2y = math.fsum(W * rw * nu * (K2 * h) ** 2)
        S1 = math.fsum(W * rw * nu * (K1 * h))
        lam0, th = 0.5 * (p.lam + p.lam_neg), 0.5 * (p.lam_neg - p.lam)
        a2 = 2.0 - 2.0 * s

        def radial_c2(t):
            # int_0^{r R(t)} C e^{-mu q} q^{1 - 2s} dq along the direction t
            mu, R = lam0 - th * math.cos(t), r * _Rtheta(t)
            if mu == 0.0:
                return R ** a2 / a2
            return mu ** (-a2) * sp.gammainc(a2, mu * R) * sp.gamma(a2)

        def radial_t(t):
            mu, R = lam0 - th * math.cos(t), LW * _Rtheta(t)
            if mu == 0.0:
                return R ** (-2.0 * s) / (2.0 * s)
            v, _ = integrate.quad(lambda q: np.exp(-mu * q) * q ** (-1.0 - 2.0 * s), R, np.inf,
                                  epsabs=0.0, epsrel=1e-13, limit=400)
            return v

        C2 = C * _quad_theta(lambda t: math.cos(t) ** 2 * radial_c2(t))
        C2y = C * _quad_theta(lambda t: math.sin(t) ** 2 * radial_c2(t))
        T = C * _quad_theta(radial_t)
        return dict(S0=S0, S2=S2, C2=C2, T=T, S1=S1, S2y=S2y, C2y=C2y, h=h, NW=NW, m=m, r=r, LW=LW)
    if d == 1:
        kk = k[nz]
        w = _trap_w(kk, NW, h)
        nu = kernel_nu(p, np.abs(kk) * h)
        S0 = math.fsum(w * nu)
        S2 = math.fsum(w * _rho_w(kk, m) * nu * (kk * h) ** 2)
        if lam == 0.0:
            C2 = 2.0 * C * r ** (2.0 - 2.0 * s) / (2.0 - 2.0 * s)
            T = C * LW ** (-2.0 * s) / s
        else:
            a2 = 2.0 - 2.0 * s
            C2 = 2.0 * C * lam ** (-a2) * sp.gammainc(a2, lam * r) * sp.gamma(a2)
            val, _ = integrate.quad(lambda y: np.exp(-lam * y) * y ** (-1.0 - 2.0 * s),
                                    LW, np.inf, epsabs=0.0, epsrel=1e-13, limit=400)
            T = 2.0 * C * val
    else:
        K1, K2 = np.meshgrid(k, k, indexing="ij")
        K1 = K1.ravel(); K2 = K2.ravel()
        nz2 = (K1 != 0) | (K2 != 0)
        K1 = K1[nz2]; K2 = K2[nz2]
        W = _trap_w(K1, NW, h) * _trap_w(K2, NW, h)
        rr = np.hypot(K1 * h, K2 * h)
        nu = kernel_nu(p, rr)
        S0 = math.fsum(W * nu)
        S2 = math.fsum(W * _rho_w(K1, m) * _rho_w(K2, m) * nu * (K1 * h) ** 2)
        if lam == 0.0:
            C2 = C * r ** (2.0 - 2.0 * s) / (2.0 - 2.0 * s) * _quad_theta(
                lambda t: math.cos(t) ** 2 * _Rtheta(t) ** (2.0 - 2.0 * s))
            T = C * LW ** (-2.0 * s) / (2.0 * s) * _quad_theta(
                lambda t: _Rtheta(t) ** (-2.0 * s))
        else:
            a2 = 2.0 - 2.0 * s

            def inner_c2(t):
                R = r * _Rtheta(t)
                return math.cos(t) ** 2 * lam ** (-a2) * sp.gammainc(a2, lam * R) * sp.gamma(a2)

            def inner_t(t):
                R = LW * _Rtheta(t)
                v, _ = integrate.quad(lambda q: np.exp(-lam * q) * q ** (-1.0 - 2.0 * s),
                                      R, np.inf, epsabs=0.0, epsrel=1e-13, limit=400)
                return v

            C2 = C * _quad_theta(inner_c2)
            T = C * _quad_theta(inner_t)
    return dict(S0=S0, S2=S2, C2=C2, T=T, h=h, NW=NW, m=m, r=r, LW=LW)


# ---------------------------------------------------------------------------
# Dense generator, row by row
# ---------------------------------------------------------------------------
def generator_row(p: Problem, i: int, consts: dict | None = None) -> np.ndarray:
    """Row i of the dense generator G (length N) for the zero-exterior box.

    Off-diagonal: the trapezoid jump entry W_k nu(kh) for every in-domain
    offset k (Sec. 4: far entries stay nu_j h), plus the local terms on the
    nearest neighbours: (C2-S2)/(2h^2) from equ:I1approx/equ:I3approx,
    a/h^2 (diffusion) and +-b/(2h) (central drift).
    Diagonal: -S0 - T (equ:I1approx, equ:I2approx), -d (C2-S2)/h^2 from the
    local Laplacian, -2 d a/h^2, and c.
    """
    if consts is None:
        consts = quadrature_constants(p)
    h = consts["h"]
    n, d = p.n, p.dim
    N = p.N
    row = np.zeros(N, dtype=np.float64)
    beta = 0.5 * (consts["C2"] - consts["S2"])
    if d == 1:
        j = np.arange(n)
        k = j - i
        if p.jumps:
            off = k != 0
            if p.lam_neg is None:
                row[off] = h * kernel_nu(p, np.abs(k[off]) * h)
            else:
                row[off] = h * kernel_nu_signed(p, k[off] * h)
        # the u' term of equ:I1approx: -S1 u'(x_i) by the central difference
        s1 = consts.get("S1", 0.0)
        for kk, sgn in ((-1, -1.0), (1, 1.0)):
            jj = i + kk
            if 0 <= jj < n:
                row[jj] += (beta + p.a) / h ** 2 + sgn * (p.b[0] - s1) / (2.0 * h)
        row[i] = -consts["S0"] - consts["T"] - 2.0 * (beta + p.a) / h ** 2 + p.c
        return row
    # 2D, index = p1*n + q1 (first coordinate slowest).  An asymmetric
    # measure has its own u'' coefficient per axis and the u' sum S1 of the
    # first axis as a drift (symmetric: the same beta twice, S1 = 0)
    p1, q1 = divmod(i, n)
    P, Q = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    K1 = (P - p1).ravel(); K2 = (Q - q1).ravel()
    if p.jumps:
        off = (K1 != 0) | (K2 != 0)
        if p.lam_neg is None:
            row[off] = h * h * kernel_nu(p, np.hypot(K1[off] * h, K2[off] * h))
        else:
            row[off] = h * h * kernel_nu_tilted(p, K1[off] * h, K2[off] * h)
    betas = (beta, 0.5 * (consts["C2y"] - consts["S2y"]) if "C2y" in consts else beta)
    drift = (p.b[0] - consts.get("S1", 0.0), p.b[1])
    for axis in (0, 1):
        for sgn in (-1, 1):
            pp, qq = p1 + (sgn if axis == 0 else 0), q1 + (sgn if axis == 1 else 0)
            if 0 <= pp < n and 0 <= qq < n:
                row[pp * n + qq] += (betas[axis] + p.a) / h ** 2 + sgn * drift[axis] / (2.0 * h)
    if "C2y" in consts:
        row[i] = (-consts["S0"] - consts["T"] - 2.0 * (betas[0] + p.a) / h ** 2 - 2.0 * (betas[1] + p.a) / h ** 2
                  + p.c)
    else:
        row[i] = -consts["S0"] - consts["T"] - 4.0 * (beta + p.a) / h ** 2 + p.c
    return row


def generator_dense(p: Problem) -> np.ndarray:
    """The full N x N generator, stacked from generator_row."""
    consts = quadrature_constants(p)
    G = np.empty((p.N, p.N), dtype=np.float64)
    for i in range(p.N):
        G[i] = generator_row(p, i, consts)
    return G


def variable_order_generator(p: Problem, mask=None, s_field=None) -> np.ndarray:
    """Generator of a variable jump index on a masked grid (Sec. 5.4,
    eq. equ:2dmodel: -(-Delta)^{s(x)} on the L-shaped domain, discretised
    row by row as in Sec. 4).

    The unknowns are the grid points the mask keeps (mask None: all), in
    grid order.  The row of the unknown at grid point g, whose jump index is
    s_g, is row g of the box generator of the same problem with s = s_g
    (kernel constant c_{d,s_g} when p.C is None) restricted to the columns
    of the unknowns: u = 0 on the grid points the mask drops, as outside
    the box, and the diagonal keeps the whole-lattice sums of that row's
    kernel.  s_field: one jump index per unknown (None: p.s everywhere)."""
    full = p.n if p.dim == 1 else p.n * p.n
    idx = np.arange(full) if mask is None else np.flatnonzero(np.asarray(mask).reshape(-1))
    svals = np.full(len(idx), p.s) if s_field is None else np.asarray(s_field, dtype=np.float64)
    if svals.shape != (len(idx),):
        raise ValueError("s_field holds one value per unknown")
    G = np.empty((len(idx), len(idx)), dtype=np.float64)
    consts = {}
    for r, g in enumerate(idx):
        s = float(svals[r])
        q = replace(p, s=s)
        if s not in consts:
            consts[s] = quadrature_constants(q)
        G[r] = generator_row(q, int(g), consts[s])[idx]
    return G


# ---------------------------------------------------------------------------
# Non-zero exterior (Sec. 4: the window terms that reach outside the box)
# ---------------------------------------------------------------------------
def exterior_forcing(p: Problem, u_ext: np.ndarray) -> np.ndarray:
    """The generator's action on exterior values, 1D: with u = u_ext outside
    the box, row i of the scheme (equ:I1approx - equ:I3approx) also takes
    the window offsets k (|k| <= NW = n + 1) whose point x_i + kh lies
    outside, each with its trapezoid weight W_k nu(kh), and the local terms
    (diffusion, drift, the u'' and u' corrections) on the exterior
    neighbours x_{-1} = lo and x_n = hi.  u_ext: the NW values left of the
    box (lattice indices -NW .. -1, ascending) followed by the NW values
    right of it (indices n .. 2n).  Returns g (length n) such that the
    scheme on the box with this exterior is G u + g.  The far field beyond
    the window (|y| > L_W) is not included: its integral of u_ext is the
    caller's (its -u T part is in the diagonal of G).  2D: see
    _exterior_forcing_2d."""
    if p.dim == 2:
        return _exterior_forcing_2d(p, u_ext)
    c = quadrature_constants(p)
    h, NW, n = c["h"], c["NW"], p.n
    beta = 0.5 * (c["C2"] - c["S2"])
    s1 = c.get("S1", 0.0)
    u_ext = np.asarray(u_ext, dtype=np.float64)
    if u_ext.shape != (2 * NW,):
        raise ValueError("u_ext holds 2 (n + 1) values")
    g = np.zeros(n)
    for i in range(n):
        acc = 0.0
        for q in range(2 * NW):
            j = q - NW if q < NW else n + (q - NW)      # lattice index of the exterior point
            k = j - i
            if abs(k) > NW:
                continue
            w = 0.5 * h if abs(k) == NW else h
            nu = (kernel_nu_signed(p, k * h) if p.lam_neg is not None else kernel_nu(p, abs(k) * h))
            v = w * float(nu)
            if k == -1:
                v += (beta + p.a) / h ** 2 - (p.b[0] - s1) / (2.0 * h)
            if k == 1:
                v += (beta + p.a) / h ** 2 + (p.b[0] - s1) / (2.0 * h)
            acc += v * u_ext[q]
        g[i] = acc
    return g


def far_field(p: Problem, u_ext: np.ndarray, next_: int, tail_left: float, tail_right: float) -> np.ndarray:
    """The far-field term f^{L_W} of equ:I2approx (eq. equ:fxy) for an
    exterior given on an extended lattice, 1D: row i takes
    int_{|y| > L_W} u_ext(x_i + y) nu(y) dy by the trapezoid rule on the
    lattice offsets k = NW .. next_ (NW = n + 1; weights h, h/2 at both
    ends; nothing when next_ = NW), plus, beyond next_ h, the constant
    tail_right (y > 0) or tail_left (y < 0) times the exact integral of nu
    over that half-line (adaptive quadrature).  u_ext: next_ values left of
    the box (lattice indices -next_ .. -1, ascending), then next_ right of
    it (indices n .. n + next_ - 1)."""
    if p.dim == 2:
        return _far_field_2d(p, u_ext, next_, tail_left, tail_right)
    c = quadrature_constants(p)
    h, NW, n = c["h"], c["NW"], p.n
    if next_ < NW:
        raise ValueError("next_ must be at least n + 1")
    u_ext = np.asarray(u_ext, dtype=np.float64)
    if u_ext.shape != (2 * next_,):
        raise ValueError("u_ext holds 2 next_ values")
    left, right = u_ext[:next_], u_ext[next_:]

    def nu(y):
        return float(kernel_nu_signed(p, y) if p.lam_neg is not None else kernel_nu(p, abs(y)))

    def tail(sign):
        val, _ = integrate.quad(lambda y: nu(sign * y), next_ * h, np.inf, epsabs=0.0, epsrel=1e-13, limit=400)
        return val

    tp, tm = tail(1.0), tail(-1.0)
    f = np.zeros(n)
    for i in range(n):
        acc = 0.0
        if next_ > NW:
            for k in range(NW, next_ + 1):
                w = 0.5 * h if k in (NW, next_) else h
                acc += w * nu(k * h) * right[i + k - n]          # lattice index i + k >= n
                acc += w * nu(-k * h) * left[i - k + next_]      # lattice index i - k <= -1
        f[i] = acc + tail_right * tp + tail_left * tm
    return f


def _exterior_forcing_2d(p: Problem, u_ext: np.ndarray) -> np.ndarray:
    """2D: u_ext holds the values on the extended lattice of indices
    -NW .. n - 1 + NW per axis ((n + 2 NW)^2 values, first coordinate
    slowest; the n^2 interior entries are ignored).  Row (p1, q1) takes every
    exterior lattice point of its window (|k|_inf <= NW) with the trapezoid
    weights W_k1 W_k2 and the row's kernel, and the local terms (diffusion,
    the u'' correction of its axis, the drift and an asymmetric measure's
    u' sum) on its exterior nearest neighbours."""
    c = quadrature_constants(p)
    h, NW, n = c["h"], c["NW"], p.n
    side = n + 2 * NW
    u_ext = np.asarray(u_ext, dtype=np.float64)
    if u_ext.shape != (side * side,):
        raise ValueError("u_ext holds (n + 2 (n + 1))^2 values")
    U = u_ext.reshape(side, side)
    betas = (0.5 * (c["C2"] - c["S2"]), 0.5 * (c["C2y"] - c["S2y"]) if "C2y" in c else 0.5 * (c["C2"] - c["S2"]))
    drift = (p.b[0] - c.get("S1", 0.0), p.b[1])
    w1 = lambda k: 0.5 * h if abs(k) == NW else h
    g = np.zeros(n * n)
    for p1 in range(n):
        for q1 in range(n):
            acc = 0.0
            for k1 in range(-NW, NW + 1):
                a1 = p1 + k1
                for k2 in range(-NW, NW + 1):
                    a2 = q1 + k2
                    if 0 <= a1 < n and 0 <= a2 < n:
                        continue              # interior point
                    if p.jumps:
                        if p.lam_neg is None:
                            nu = float(kernel_nu(p, math.hypot(k1 * h, k2 * h)))
                        else:
                            nu = float(kernel_nu_tilted(p, k1 * h, k2 * h))
                        v = w1(k1) * w1(k2) * nu
                    else:
                        v = 0.0
                    if abs(k1) + abs(k2) == 1:
                        ax = 0 if k1 != 0 else 1
                        sg = k1 if k1 != 0 else k2
                        v += (betas[ax] + p.a) / h ** 2 + sg * drift[ax] / (2.0 * h)
                    acc += v * U[a1 + NW, a2 + NW]
            g[p1 * n + q1] = acc
    return g


def _far_field_2d(p: Problem, u_ext, next_: int, tail_left: float, tail_right: float) -> np.ndarray:
    """2D far field: u_ext holds the extended lattice of indices
    -next_ .. n - 1 + next_ per axis ((n + 2 next_)^2 values, first coordinate
    slowest; entries inside the window of every row are not read).  Row i
    takes the product trapezoid rule over the square |k|_inf <= next_ (weights
    h, h/2 at |k_a| = next_) less the window's (|k|_inf <= NW, h/2 at
    |k_a| = NW), so only points with |k|_inf >= NW enter, all exterior; beyond
    the square the constant tail_right (y1 > 0) or tail_left (y1 < 0) times
    the measure of that half of the region |y|_inf > next_ h (adaptive
    quadrature in polar coordinates)."""
    c = quadrature_constants(p)
    h, NW, n = c["h"], c["NW"], p.n
    if next_ < NW:
        raise ValueError("next_ must be at least n + 1")
    side = n + 2 * next_
    U = np.asarray(u_ext, dtype=np.float64).reshape(side, side)
    k = np.arange(-next_, next_ + 1)
    K1, K2 = np.meshgrid(k, k, indexing="ij")
    wb = np.where(np.abs(k) == next_, 0.5 * h, h)
    ww = np.where(np.abs(k) == NW, 0.5 * h, np.where(np.abs(k) < NW, h, 0.0))
    W = np.outer(wb, wb) - np.outer(ww, ww)
    W[(np.abs(K1) < NW) & (np.abs(K2) < NW)] = 0.0      # the window's inside: nothing
    nz = (K1 != 0) | (K2 != 0)
    nu = np.zeros_like(W)
    if p.lam_neg is None:
        nu[nz] = kernel_nu(p, np.hypot(K1[nz] * h, K2[nz] * h))
    else:
        nu[nz] = kernel_nu_tilted(p, K1[nz] * h, K2[nz] * h)
    coef = W * nu
    R = next_ * h

    def half(sign):
        def radial(phi):
            cs, sn = math.cos(phi), math.sin(phi)
            r0 = R / max(abs(cs), abs(sn))
            if p.lam_neg is None:
                f = lambda r: float(kernel_nu(p, r)) * r
            else:
                f = lambda r: float(kernel_nu_tilted(p, r * cs, r * sn)) * r
            return integrate.quad(f, r0, np.inf, epsabs=0.0, epsrel=1e-13, limit=400)[0]
        # y1 > 0: phi in (-pi/2, pi/2), octants split at the square's corners
        base = -math.pi / 2 if sign > 0 else math.pi / 2
        return sum(integrate.quad(radial, base + q * math.pi / 4, base + (q + 1) * math.pi / 4, epsabs=0.0,
                                  epsrel=1e-12, limit=200)[0] for q in range(4))

    tp, tm = half(1.0), half(-1.0)
    f = np.zeros(n * n)
    for p1 in range(n):
        for q1 in range(n):
            blk = U[p1:p1 + 2 * next_ + 1, q1:q1 + 2 * next_ + 1]
            f[p1 * n + q1] = float(np.sum(coef * np.where(W != 0.0, blk, 0.0)))
    return f + tail_right * tp + tail_left * tm


# ---------------------------------------------------------------------------
# Fixed-rank Taylor factors of the Gaussian kernel (Sec. 3.3)
# ---------------------------------------------------------------------------
def taylor_terms(dim: int, rank: int) -> list:
    """Exponents of the first `rank` terms of the expansion: 1D n = 0, 1,
    ...; 2D the products (n1, n2) of the 1D series in order of total degree
    n1 + n2, then of n2."""
    if dim == 1:
        return [(n,) for n in range(rank)]
    out, deg = [], 0
    while len(out) < rank:
        for n2 in range(deg + 1):
            if len(out) < rank:
                out.append((deg - n2, n2))
        deg += 1
    return out


def taylor_factors(p: Problem, rows, cols, rank: int):
    """U (m x rank), V (n x rank) with U V^T approximating the generator's
    block h^d nu(x_j - x_i) (i in rows, j in cols) for the Gaussian kernel,
    from the Taylor expansion about the centre xbar of the row points'
    bounding box (Sec. 3.3): with t0 = x - xbar and t = y - xbar per axis,
    alpha_n(t0) = (2 eps2)^n exp(-eps2 t0^2) t0^n / n! and
    beta_n(t) = exp(-eps2 t^2) t^n, so that exp(-eps2 (x - y)^2) is
    sum_n alpha_n(t0) beta_n(t); in 2D a term is the product of one 1D term
    per axis.  U carries the factor h^d C."""
    pts = grid(p)
    X = pts[np.asarray(rows)]
    Y = pts[np.asarray(cols)]
    xbar = 0.5 * (X.min(axis=0) + X.max(axis=0))
    t0 = X - xbar
    t = Y - xbar
    h = h_of(p)
    e = p.eps2
    terms = taylor_terms(p.dim, rank)
    U = np.empty((len(X), rank))
    V = np.empty((len(Y), rank))
    for q, ns in enumerate(terms):
        a = np.full(len(X), (h ** p.dim) * p.Cval)
        b = np.ones(len(Y))
        for ax, n in enumerate(ns):
            a = a * (2.0 * e) ** n * np.exp(-e * t0[:, ax] ** 2) * t0[:, ax] ** n / math.factorial(n)
            b = b * np.exp(-e * t[:, ax] ** 2) * t[:, ax] ** n
        U[:, q] = a
        V[:, q] = b
    return U, V


# ---------------------------------------------------------------------------
# Crank-Nicolson (Sec. 3.2, eq. equ:scheme) with trapezoidal forcing
# ---------------------------------------------------------------------------
def cn_matrices(G: np.ndarray, dt: float):
    """M = I - dt/2 G (left side), Mp = I + dt/2 G (right side)."""
    I = np.eye(G.shape[0])
    return I - 0.5 * dt * G, I + 0.5 * dt * G


@dataclass
class CNResult:
    u: np.ndarray
    norms: list = field(default_factory=list)


def cn_run(G: np.ndarray, dt: float, steps: int, u0: np.ndarray,
           g: np.ndarray | None = None, phi: np.ndarray | None = None,
           keep_norms: bool = False) -> CNResult:
    """u^{n+1} = M^{-1} (Mp u^n + dt/2 (f^n + f^{n+1})),  f^n = phi[n] g.

    M is factored once with LAPACK getrf (partial pivoting); each step is one
    dense product and one getrs.
    """
    M, Mp = cn_matrices(G, dt)
    lu = sla.lu_factor(M)
    u = np.array(u0, dtype=np.float64, copy=True)
    norms = [float(np.linalg.norm(u))] if keep_norms else []
    for n in range(steps):
        rhs = Mp @ u
        if g is not None:
            rhs = rhs + 0.5 * dt * (phi[n] + phi[n + 1]) * g
        u = sla.lu_solve(lu, rhs)
        if keep_norms:
            norms.append(float(np.linalg.norm(u)))
    return CNResult(u=u, norms=norms)


# ---------------------------------------------------------------------------
# Steady problems (Sec. 5.1 preconditioned solves; Sec. 5.3 fractional Poisson)
# ---------------------------------------------------------------------------
def steady_solve(G: np.ndarray, shift: float, f: np.ndarray) -> np.ndarray:
    """u with (shift I - G) u = f, by dense LU with partial pivoting
    (LAPACK getrf/getrs).  With shift = 0 and the fractional generator this
    is (-Delta)^s u = f with zero exterior (Sec. 5.3)."""
    A = shift * np.eye(G.shape[0]) - G
    return sla.lu_solve(sla.lu_factor(A), f)


def steady_residual(G: np.ndarray, shift: float, u: np.ndarray, f: np.ndarray) -> float:
    """||(shift I - G) u - f||_2 / ||f||_2, the relative error the paper
    tracks over the iterations of a preconditioned solve (Sec. 5.4,
    eq. equ:relative_error)."""
    r = shift * u - G @ u - f
    return float(np.linalg.norm(r) / np.linalg.norm(f))


def fractional_poisson_exact(d: int, s: float, x: np.ndarray) -> np.ndarray:
    """(1 - |x|^2)_+^s / K(d, s): the solution of (-Delta)^s u = 1 on the
    unit ball with zero exterior, K = ball_const (Sec. 5.3; see the reading
    of its constant in the module docstring).  x: points, shape (N, d)."""
    r2 = np.sum(np.asarray(x, dtype=np.float64).reshape(len(x), -1) ** 2, axis=1)
    return np.maximum(1.0 - r2, 0.0) ** s / ball_const(d, s)


# ---------------------------------------------------------------------------
# Crank-Nicolson at full size with a single N x N array (Sec. 3.2, equ:scheme)
# ---------------------------------------------------------------------------
def _getrf_in_place(A: np.ndarray):
    """LAPACK getrf (partial pivoting) of the column-major matrix whose
    memory is the row-major array A (that is, of A^T), overwriting A.

    The call goes to the getrf of torch's CPU LAPACK (MKL) with its output
    aliased to its input, which factors in place.  The OpenBLAS getrf that
    scipy links faults (a write past one of its packing buffers) on a
    65536 x 65536 matrix.  Returns (lu, piv) in scipy's lu_factor form:
    lu the column-major factors (a view of A's memory), piv 0-based."""
    import torch
    T = torch.from_numpy(A)                         # shares A's memory
    LU = T.T                                        # column-major view of A^T
    piv = torch.empty(A.shape[0], dtype=torch.int32)
    info = torch.empty((), dtype=torch.int32)
    torch.linalg.lu_factor_ex(LU, out=(LU, piv, info))
    if LU.data_ptr() != T.data_ptr():
        raise RuntimeError("getrf copied the matrix; the lean path needs it in place")
    if int(info) != 0:
        raise RuntimeError(f"getrf: info = {int(info)}")
    return A.T, piv.numpy().astype(np.int64) - 1


def cn_run_lean(p: Problem, dt: float, steps: int, u0: np.ndarray,
                g: np.ndarray | None = None, phi: np.ndarray | None = None,
                keep_norms: bool = False, log=None) -> CNResult:
    """The recursion of ``cn_run`` for N where two dense N x N arrays do not
    fit in host memory (N = 65536 needs 34 GB per array).

    The rows of M = I - dt/2 G are written, one generator row at a time, into
    one row-major array.  Read in column-major order the same memory holds
    M^T, which LAPACK getrf factors in place (``_getrf_in_place``):
    M^T = P L U.  Hence
    M = U^T L^T P^T, and each step is the plain recursion

        rhs     = 2 u^n - M u^n + dt/2 (f^n + f^{n+1})     (M_+ = 2 I - M)
        u^{n+1} = M^{-1} rhs

    with M u^n = U^T (L^T (P^T u^n)) formed by two BLAS triangular products
    on the factors, and M^{-1} rhs by the transposed getrs solve.

    Returns a CNResult whose ``timings`` attribute holds the seconds spent in
    assembly, factorisation and the step loop.
    """
    import time
    from scipy.linalg import blas

    say = log if log is not None else (lambda msg: None)
    N = p.N
    t0 = time.perf_counter()
    consts = quadrature_constants(p)
    A = np.empty((N, N), dtype=np.float64)          # row-major: row i of M
    for i in range(N):
        row = generator_row(p, i, consts)
        row *= -0.5 * dt
        row[i] += 1.0
        A[i] = row
        if (i + 1) % 8192 == 0:
            say(f"assembled {i + 1}/{N} rows")
    t1 = time.perf_counter()
    lu, piv = _getrf_in_place(A)
    t2 = time.perf_counter()
    say(f"factored in {t2 - t1:.1f}s")

    def m_times(v):
        w = np.array(v, dtype=np.float64, copy=True)
        for i in range(N):                          # P^T v: the interchanges in order
            j = piv[i]
            if j != i:
                w[i], w[j] = w[j], w[i]
        w = blas.dtrmv(lu, w, lower=1, trans=1, diag=1)     # L^T (unit diagonal)
        return blas.dtrmv(lu, w, lower=0, trans=1)          # U^T

    u = np.array(u0, dtype=np.float64, copy=True)
    norms = [float(np.linalg.norm(u))] if keep_norms else []
    for n in range(steps):
        rhs = 2.0 * u - m_times(u)
        if g is not None:
            rhs = rhs + 0.5 * dt * (phi[n] + phi[n + 1]) * g
        u = sla.lu_solve((lu, piv), rhs, trans=1, check_finite=False)
        if keep_norms:
            norms.append(float(np.linalg.norm(u)))
        if (n + 1) % 10 == 0:
            say(f"step {n + 1}/{steps} |u| {np.linalg.norm(u):.15e} "
                f"{(time.perf_counter() - t2) / (n + 1):.3f}s/step")
    t3 = time.perf_counter()
    res = CNResult(u=u, norms=norms)
    res.timings = dict(assembly_s=t1 - t0, factor_s=t2 - t1, steps_s=t3 - t2)
    return res
