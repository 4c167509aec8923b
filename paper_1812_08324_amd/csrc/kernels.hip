// HIP kernels for gfx950 (CDNA4, 64-wide wavefronts) of the H-matrix
// Crank-Nicolson library.  Host-side launchers are at the end of the file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "hl_jobs.h"
#include "hl_kernels.h"

namespace hl {

typedef double double4v __attribute__((ext_vector_type(4)));

#define HL_BLOCK 256

// ---------------------------------------------------------------------------
// double-double helpers (error-free transformations; FMA for products).
// Every helper forbids floating-point contraction: a product rounded in one
// helper must not be fused into an addition of another after inlining (an
// fma there would add the exact product while the low part assumes the
// rounded one, and the pair would lose every bit beyond FP64).
// ---------------------------------------------------------------------------
struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
#pragma clang fp contract(off)
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ __forceinline__ dd quick_two_sum(double a, double b) {
#pragma clang fp contract(off)
  double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
#pragma clang fp contract(off)
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
#pragma clang fp contract(off)
  double p = a.hi * b.hi;
  double e = fma(a.hi, b.hi, -p);
  e += a.hi * b.lo + a.lo * b.hi;
  return quick_two_sum(p, e);
}
__device__ __forceinline__ dd dd_mul_d(double a, double b) {
#pragma clang fp contract(off)
  double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_div(dd a, dd b) {
#pragma clang fp contract(off)
  double q1 = a.hi / b.hi;
  dd r = dd_add(a, dd_neg(dd_mul({q1, 0.0}, b)));
  double q2 = r.hi / b.hi;
  r = dd_add(r, dd_neg(dd_mul({q2, 0.0}, b)));
  double q3 = r.hi / b.hi;
  dd q = quick_two_sum(q1, q2);
  return dd_add(q, {q3, 0.0});
}
__device__ __forceinline__ dd dd_sqrt(dd a) {
#pragma clang fp contract(off)
  if (a.hi <= 0.0) return {0.0, 0.0};
  double x = sqrt(a.hi);
  dd xx = dd_mul_d(x, x);
  dd r = dd_add(a, dd_neg(xx));
  return quick_two_sum(x, r.hi / (2.0 * x));
}

// ---------------------------------------------------------------------------
// block reductions
// ---------------------------------------------------------------------------
__device__ __forceinline__ double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the block (blockDim.x == 256); result valid in every thread.
__device__ double block_sum(double v, double* red) {
  v = warp_sum(v);
  int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  double s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

// Maximum over the block (blockDim.x == 256); result valid in every thread.
__device__ double block_max(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return m;
}

// ---------------------------------------------------------------------------
// kernel of the jump measure and quadrature constants (Sec. 4)
// ---------------------------------------------------------------------------
// the tempered kernel at distance r with jump index s and constant C
__device__ __forceinline__ double nu_sc(const ProblemDev& P, double r, double s, double C) {
  return C * exp(-P.lam * r) / pow(r, (double)P.dim + 2.0 * s);
}
__device__ __forceinline__ double nu_at(const ProblemDev& P, double r) {
  if (P.kernel == HLEVY_KERNEL_GAUSSIAN) return P.C * exp(-P.eps2 * r * r);
  return nu_sc(P, r, P.s, P.C);
}
// nu at the 1D jump y = k h (k != 0): the asymmetric kernel takes the rate
// of its side, every other kernel is even
__device__ __forceinline__ double nu_jump1(const ProblemDev& P, int k) {
  const double r = fabs((double)k) * P.h;
  if (P.kernel == HLEVY_KERNEL_TEMPERED_ASYM)
    return P.C * exp(-(k > 0 ? P.lam : P.lam_neg) * r) / pow(r, 1.0 + 2.0 * P.s);
  return nu_at(P, r);
}

// 2D asymmetric tempered kernel at the jump (k1 h, k2 h): the symmetric
// kernel tilted along the first axis, C exp(-lam0 |y| + theta y1) /
// |y|^{2+2s}, lam0 = (lam + lam_neg)/2, theta = (lam_neg - lam)/2 (rates lam
// and lam_neg along the first axis, as in 1D)
__device__ __forceinline__ double nu_tilt2(const ProblemDev& P, int k1, int k2) {
  const double r = P.h * sqrt((double)k1 * k1 + (double)k2 * k2);
  const double lam0 = 0.5 * (P.lam + P.lam_neg), th = 0.5 * (P.lam_neg - P.lam);
  return P.C * exp(-lam0 * r + th * (k1 * P.h)) / pow(r, 2.0 + 2.0 * P.s);
}

// lower incomplete gamma gamma(a, x) by its power series (x moderate)
__device__ double lower_gamma(double a, double x) {
  if (x <= 0.0) return 0.0;
  double term = 1.0 / a, sum = term;
  for (int k = 1; k < 400; ++k) {
    term *= x / (a + k);
    sum += term;
    if (fabs(term) < 1e-17 * fabs(sum)) break;
  }
  return sum * exp(a * log(x) - x);
}

// exponential integral E1(x) = Gamma(0, x), x > 0: the power series
// -gamma_E - ln x - sum_k (-x)^k / (k k!) below 1, above it the continued
// fraction 1 / (x + 1 - 1 / (x + 3 - 4 / (x + 5 - ...))) times e^{-x}
// (modified Lentz)
__device__ double expint_e1(double x) {
  if (x <= 1.0) {
    double sum = 0.0, term = 1.0;
    for (int k = 1; k < 60; ++k) {
      term *= -x / k;
      const double add = term / k;
      sum += add;
      if (fabs(add) < 1e-17 * fabs(sum)) break;
    }
    return -0.57721566490153286061 - log(x) - sum;
  }
  double b = x + 1.0, c = 1e300, d = 1.0 / b, f = d;
  for (int i = 1; i < 300; ++i) {
    const double an = -(double)i * i;
    b += 2.0;
    d = an * d + b;
    if (fabs(d) < 1e-300) d = 1e-300;
    c = b + an / c;
    if (fabs(c) < 1e-300) c = 1e-300;
    d = 1.0 / d;
    const double del = c * d;
    f *= del;
    if (fabs(del - 1.0) < 1e-16) break;
  }
  return f * exp(-x);
}

// upper incomplete gamma Gamma(a, x) for a in (-2, 1], x > 0 (a = 0 and
// a = -1, i.e. s = 1/2, go through E1)
__device__ double upper_gamma(double a, double x) {
  if (a == 0.0) return expint_e1(x);
  if (a > 0.0) {
    if (x > 30.0) {
      // continued fraction (Lentz) for large x
      double b = x + 1.0 - a, c = 1e300, d = 1.0 / b, f = d;
      for (int i = 1; i < 300; ++i) {
        double an = -i * (i - a);
        b += 2.0;
        d = an * d + b;
        if (fabs(d) < 1e-300) d = 1e-300;
        c = b + an / c;
        if (fabs(c) < 1e-300) c = 1e-300;
        d = 1.0 / d;
        double del = d * c;
        f *= del;
        if (fabs(del - 1.0) < 1e-16) break;
      }
      return exp(a * log(x) - x) * f;
    }
    return tgamma(a) - lower_gamma(a, x);
  }
  // Gamma(a, x) = (Gamma(a+1, x) - x^a e^{-x}) / a
  return (upper_gamma(a + 1.0, x) - exp(a * log(x) - x)) / a;
}

// Gauss-Legendre node i of n on [-1, 1] by Newton's method on P_n
__device__ void gauss_legendre(int n, int i, double* x, double* w) {
  double z = cos(M_PI * (i + 0.75) / (n + 0.5));
  double pp = 0.0;
  for (int it = 0; it < 100; ++it) {
    double p1 = 1.0, p2 = 0.0;
    for (int j = 1; j <= n; ++j) {
      double p3 = p2;
      p2 = p1;
      p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
    }
    pp = n * (z * p1 - p2) / (z * z - 1.0);
    double z1 = z;
    z = z1 - p1 / pp;
    if (fabs(z - z1) < 1e-16) break;
  }
  *x = z;
  *w = 2.0 / ((1.0 - z * z) * pp * pp);
}

// out = {S0, S2, C2, T, S1} for the jump index s and kernel constant C
// (the tempered family; the Gaussian kernel reads P).  One block.
//   S0 = sum' W_k nu(kh) over the window |k|_inf <= NW = n + 1 (L_W = (n+1)h),
//        trapezoid weights h (h/2 on the window edge) per axis;
//   S2 = sum' W_k rho_k nu(kh) (k_1 h)^2 with rho the grid window of radius
//        m = round(r0/h) (weight 1/2 on its edge);
//   C2 = int rho nu y_1^2 dy,  T = int_{|y|_inf > L_W} nu dy.
__device__ void constants_of(const ProblemDev& P, const double s_, const double C_, double* out) {
  __shared__ double red[4];
  __shared__ double glx[32], glw[32];
  if (P.kernel == HLEVY_KERNEL_GAUSSIAN) {
    // Bounded kernel (Sec. 3.2, equ:dl): the coefficient of -u_i is
    // h^d sum over the lattice without 0 of nu(kh).  The lattice sum of the
    // Gaussian factorises over the axes: theta = sum_k exp(-eps2 (kh)^2)
    // over k in Z, S0 = C h^d (theta^d - 1).  Terms below 1e-18 are dropped.
    const double h = P.h;
    const int K = (int)ceil(sqrt(41.5 / P.eps2) / h) + 1;
    double t = 0.0, tc = 0.0;
    for (int k = K - (int)threadIdx.x; k >= 1; k -= blockDim.x) {   // small terms first
      const double v = exp(-P.eps2 * (k * h) * (k * h));
      const double y = v - tc, z = t + y;
      tc = (z - t) - y;
      t = z;
    }
    const double half = block_sum(t, red) - block_sum(tc, red);   // sum over k >= 1
    if (threadIdx.x == 0) {
      const double theta = 1.0 + 2.0 * half;
      out[0] = P.dim == 1 ? P.C * h * (2.0 * half) : P.C * h * h * (theta * theta - 1.0);
      out[1] = 0.0;
      out[2] = 0.0;
      out[3] = 0.0;
      out[4] = 0.0;
    }
    return;
  }
  const int NW = P.n + 1;
  const double h = P.h;
  const int m = (int)floor(P.r0 / h + 0.5);   // nearest grid multiple, ties up
  const double r = m * h, LW = NW * h;
  double s0 = 0.0, s0c = 0.0, s2 = 0.0, s2c = 0.0;  // Neumaier-compensated partial sums
  auto acc = [](double& s, double& c, double v) {
    double t = s + v;
    if (fabs(s) >= fabs(v)) c += (s - t) + v; else c += (v - t) + s;
    s = t;
  };
  double s1 = 0.0, s1c = 0.0;   // u' sum of an asymmetric measure
  double s2y = 0.0, s2yc = 0.0; // u'' sum of the second axis (2D asymmetric)
  if (P.dim == 1 && P.kernel == HLEVY_KERNEL_TEMPERED_ASYM) {
    for (int k = 1 + threadIdx.x; k <= NW; k += blockDim.x) {
      double w = (k == NW) ? 0.5 * h : h;
      const double np = nu_jump1(P, k), nn = nu_jump1(P, -k);
      acc(s0, s0c, w * np);
      acc(s0, s0c, w * nn);
      if (k <= m) {
        double rho = (k < m) ? 1.0 : 0.5;
        acc(s2, s2c, w * rho * np * (k * h) * (k * h));
        acc(s2, s2c, w * rho * nn * (k * h) * (k * h));
        acc(s1, s1c, w * rho * (np - nn) * (k * h));
      }
    }
  } else if (P.dim == 1) {
    for (int k = 1 + threadIdx.x; k <= NW; k += blockDim.x) {
      double w = (k == NW) ? 0.5 * h : h;
      double nu = nu_sc(P, k * h, s_, C_);
      acc(s0, s0c, 2.0 * w * nu);
      if (k <= m) {
        double rho = (k < m) ? 1.0 : 0.5;
        acc(s2, s2c, 2.0 * w * rho * nu * (k * h) * (k * h));
      }
    }
  } else if (P.kernel == HLEVY_KERNEL_TEMPERED_ASYM) {
    // tilted 2D kernel: the u' sum S1 of the first axis, the u'' sums of
    // both axes (the second axis's in s2y)
    const int side = 2 * NW + 1;
    const long total = (long)side * side;
    for (long idx = threadIdx.x; idx < total; idx += blockDim.x) {
      int k1 = (int)(idx / side) - NW, k2 = (int)(idx % side) - NW;
      if (k1 == 0 && k2 == 0) continue;
      double w = ((abs(k1) == NW) ? 0.5 * h : h) * ((abs(k2) == NW) ? 0.5 * h : h);
      double nu = nu_tilt2(P, k1, k2);
      acc(s0, s0c, w * nu);
      if (abs(k1) <= m && abs(k2) <= m) {
        double rho = ((abs(k1) < m) ? 1.0 : 0.5) * ((abs(k2) < m) ? 1.0 : 0.5);
        acc(s2, s2c, w * rho * nu * (k1 * h) * (k1 * h));
        acc(s2y, s2yc, w * rho * nu * (k2 * h) * (k2 * h));
        acc(s1, s1c, w * rho * nu * (k1 * h));
      }
    }
  } else {
    const int side = 2 * NW + 1;
    const long total = (long)side * side;
    for (long idx = threadIdx.x; idx < total; idx += blockDim.x) {
      int k1 = (int)(idx / side) - NW, k2 = (int)(idx % side) - NW;
      if (k1 == 0 && k2 == 0) continue;
      double w = ((abs(k1) == NW) ? 0.5 * h : h) * ((abs(k2) == NW) ? 0.5 * h : h);
      double rr = h * sqrt((double)k1 * k1 + (double)k2 * k2);
      double nu = nu_sc(P, rr, s_, C_);
      acc(s0, s0c, w * nu);
      if (abs(k1) <= m && abs(k2) <= m) {
        double rho = ((abs(k1) < m) ? 1.0 : 0.5) * ((abs(k2) < m) ? 1.0 : 0.5);
        acc(s2, s2c, w * rho * nu * (k1 * h) * (k1 * h));
      }
    }
  }
  double S0 = block_sum(s0, red) + block_sum(s0c, red);
  double S2 = block_sum(s2, red) + block_sum(s2c, red);
  const double S1 = block_sum(s1, red) + block_sum(s1c, red);
  const double S2y = block_sum(s2y, red) + block_sum(s2yc, red);
  if (threadIdx.x < 32) gauss_legendre(32, threadIdx.x, &glx[threadIdx.x], &glw[threadIdx.x]);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double s = s_, C = C_, lam = P.lam, a2 = 2.0 - 2.0 * s;
    double C2 = 0.0, T = 0.0;
    if (P.dim == 1 && P.kernel == HLEVY_KERNEL_TEMPERED_ASYM) {
      // each side with its own rate
      for (int side = 0; side < 2; ++side) {
        const double rate = side == 0 ? lam : P.lam_neg;
        if (rate == 0.0) {
          C2 += C * pow(r, a2) / a2;
          T += C * pow(LW, -2.0 * s) / (2.0 * s);
        } else {
          C2 += C * pow(rate, -a2) * lower_gamma(a2, rate * r);
          T += C * pow(rate, 2.0 * s) * upper_gamma(-2.0 * s, rate * LW);
        }
      }
    } else if (P.kernel == HLEVY_KERNEL_TEMPERED_ASYM) {
      // tilted 2D kernel: full circle, eight octants of 32 Gauss-Legendre
      // nodes (R(phi) = 1 / max(|cos|, |sin|) is smooth inside each); along
      // phi the rate is mu = lam0 - theta cos(phi)
      const double lam0 = 0.5 * (lam + P.lam_neg), th = 0.5 * (P.lam_neg - lam);
      double cx = 0.0, cy = 0.0, tt = 0.0;
      for (int oct = 0; oct < 8; ++oct)
        for (int q = 0; q < 32; ++q) {
          const double ph = 0.125 * M_PI * (glx[q] + 1.0) + 0.25 * M_PI * oct, w = 0.125 * M_PI * glw[q];
          const double c = cos(ph), sn = sin(ph);
          const double R = 1.0 / fmax(fabs(c), fabs(sn));
          const double mu = lam0 - th * c;
          double rc, rt;
          if (mu == 0.0) {
            rc = pow(r * R, a2) / a2;
            rt = pow(LW * R, -2.0 * s) / (2.0 * s);
          } else {
            rc = pow(mu, -a2) * lower_gamma(a2, mu * r * R);
            rt = pow(mu, 2.0 * s) * upper_gamma(-2.0 * s, mu * LW * R);
          }
          cx += w * c * c * rc;
          cy += w * sn * sn * rc;
          tt += w * rt;
        }
      C2 = C * cx;
      T = C * tt;
      out[5] = S2y;
      out[6] = C * cy;
    } else if (P.dim == 1) {
      if (lam == 0.0) {
        C2 = 2.0 * C * pow(r, a2) / a2;
        T = C * pow(LW, -2.0 * s) / s;
      } else {
        C2 = 2.0 * C * pow(lam, -a2) * lower_gamma(a2, lam * r);
        T = 2.0 * C * pow(lam, 2.0 * s) * upper_gamma(-2.0 * s, lam * LW);
      }
    } else {
      // theta integrals over [0, 2 pi] reduce to 8 x [0, pi/4] with
      // R(theta) = 1/cos(theta) there; cos^2 averages to 1/2 by symmetry.
      double ic = 0.0, it = 0.0;
      for (int q = 0; q < 32; ++q) {
        double th = 0.125 * M_PI * (glx[q] + 1.0), w = 0.125 * M_PI * glw[q];
        double R = 1.0 / cos(th);
        if (lam == 0.0) {
          ic += w * pow(R, a2);
          it += w * pow(R, -2.0 * s);
        } else {
          ic += w * pow(lam, -a2) * lower_gamma(a2, lam * r * R);
          it += w * pow(lam, 2.0 * s) * upper_gamma(-2.0 * s, lam * LW * R);
        }
      }
      if (lam == 0.0) {
        C2 = C * pow(r, a2) / a2 * 4.0 * ic;
        T = C * pow(LW, -2.0 * s) / (2.0 * s) * 8.0 * it;
      } else {
        C2 = 4.0 * C * ic;
        T = 8.0 * C * it;
      }
    }
    out[0] = S0;
    out[1] = S2;
    out[2] = C2;
    out[3] = T;
    out[4] = S1;
  }
}

__global__ void __launch_bounds__(HL_BLOCK) k_constants(ProblemDev P, double* out) {
  constants_of(P, P.s, P.C, out);
}

// variable-order kernel: block q computes the constants of the q-th
// distinct jump index into out[5 q .. 5 q + 4]
__global__ void __launch_bounds__(HL_BLOCK) k_constants_var(ProblemDev P, double* out) {
  const int q = blockIdx.x;
  constants_of(P, P.var_s[q], P.var_C[q], out + 5 * (size_t)q);
}

// Generator entry G_ij (cluster-ordered i, j) from integer grid offsets.
__device__ __forceinline__ double gen_entry(const ProblemDev& P, const double* cst,
                                            const int32_t* perm, int i, int j) {
  const double h = P.h;
  const bool var = P.kernel == HLEVY_KERNEL_VARIABLE_ORDER;
  double s = P.s, C = P.C;
  if (var) {   // row i's own jump index and constants
    const int q = P.var_row[i];
    s = P.var_s[q];
    C = P.var_C[q];
    cst = P.var_cst + 5 * (size_t)q;
  }
  const double beta = 0.5 * (cst[2] - cst[1]);
  // 2D asymmetric measure: the second axis has its own u'' coefficient
  const bool asym2 = P.kernel == HLEVY_KERNEL_TEMPERED_ASYM && P.dim == 2;
  const double beta_y = asym2 ? 0.5 * (cst[6] - cst[5]) : beta;
  int k1, k2 = 0;
  if (P.dim == 1) {
    k1 = j - i;
  } else {
    int pi = perm[i], pj = perm[j];
    k1 = pj / P.n - pi / P.n;
    k2 = pj % P.n - pi % P.n;
  }
  if (k1 == 0 && k2 == 0) {
    if (asym2) return -cst[0] - cst[3] - 2.0 * (beta + P.a) / (h * h) - 2.0 * (beta_y + P.a) / (h * h) + P.c;
    return -cst[0] - cst[3] - 2.0 * P.dim * (beta + P.a) / (h * h) + P.c;
  }
  double v;
  if (P.dim == 1) {
    v = h * (var ? nu_sc(P, fabs((double)k1) * h, s, C) : nu_jump1(P, k1));
  } else if (asym2) {
    v = h * h * nu_tilt2(P, k1, k2);
  } else {
    const double rr = h * sqrt((double)k1 * k1 + (double)k2 * k2);
    v = h * h * (var ? nu_sc(P, rr, s, C) : nu_at(P, rr));
  }
  if (abs(k1) + abs(k2) == 1) {
    v += ((k1 == 0 ? beta_y : beta) + P.a) / (h * h);
    // drift by the central difference; an asymmetric measure adds -S1 (the
    // u' sum of equ:I1approx, cst[4], zero otherwise)
    const double b0 = P.kernel == HLEVY_KERNEL_TEMPERED_ASYM ? P.b0 - cst[4] : P.b0;
    if (k1 != 0) v += (k1 > 0 ? 1.0 : -1.0) * b0 / (2.0 * h);
    else v += (k2 > 0 ? 1.0 : -1.0) * P.b1 / (2.0 * h);
  }
  return v;
}

// Far-field entry (admissible blocks hold no local terms).
__device__ __forceinline__ double far_entry(const ProblemDev& P, const int32_t* perm, int i, int j) {
  int k1, k2 = 0;
  if (P.dim == 1) {
    k1 = j - i;
  } else {
    int pi = perm[i], pj = perm[j];
    k1 = pj / P.n - pi / P.n;
    k2 = pj % P.n - pi % P.n;
  }
  if (P.kernel == HLEVY_KERNEL_VARIABLE_ORDER) {   // row i's own jump index
    const int q = P.var_row[i];
    const double r = P.h * sqrt((double)k1 * k1 + (double)k2 * k2);
    return (P.dim == 1 ? P.h : P.h * P.h) * nu_sc(P, r, P.var_s[q], P.var_C[q]);
  }
  if (P.dim == 1) return P.h * nu_jump1(P, k1);
  if (P.kernel == HLEVY_KERNEL_TEMPERED_ASYM) return P.h * P.h * nu_tilt2(P, k1, k2);
  double rr = P.h * sqrt((double)k1 * k1 + (double)k2 * k2);
  return P.h * P.h * nu_at(P, rr);
}

// Non-zero exterior, 1D (Sec. 4: the window terms that reach outside the
// box).  tab[k + NW] (|k| <= NW, k != 0) is the coefficient of u(x_i + kh) in
// row i: the trapezoid jump entry W_k nu(kh) (W_k = h, h/2 at |k| = NW), plus
// on k = +-1 the local terms (diffusion and the u'' correction, the drift and
// an asymmetric measure's u' sum).
__global__ void __launch_bounds__(HL_BLOCK) k_ext_table(ProblemDev P, const double* cst, double* tab) {
  const int NW = P.n + 1;
  const int q = blockIdx.x * HL_BLOCK + threadIdx.x;
  if (q > 2 * NW) return;
  const int k = q - NW;
  if (k == 0) {
    tab[q] = 0.0;
    return;
  }
  const double h = P.h;
  double v = (abs(k) == NW ? 0.5 * h : h) * nu_jump1(P, k);
  if (abs(k) == 1) {
    const double beta = 0.5 * (cst[2] - cst[1]);
    const double b0 = P.kernel == HLEVY_KERNEL_TEMPERED_ASYM ? P.b0 - cst[4] : P.b0;
    v += (beta + P.a) / (h * h) + (k > 0 ? 1.0 : -1.0) * b0 / (2.0 * h);
  }
  tab[q] = v;
}
// g[i] = sum over the exterior lattice points within the window of row i of
// tab[j - i + NW] u_ext: u_ext[0 .. NW) are lattice indices -NW .. -1,
// u_ext[NW .. 2 NW) indices n .. 2n.  One block per row, fixed-order sum.
__global__ void __launch_bounds__(HL_BLOCK) k_ext_apply(const double* tab, const double* u_ext, int n,
                                                        double* g) {
  __shared__ double red[4];
  const int NW = n + 1, i = blockIdx.x;
  double acc = 0.0;
  // left: j = q - NW >= i - NW, i.e. q >= i
  for (int q = i + threadIdx.x; q < NW; q += HL_BLOCK) acc += tab[q - NW - i + NW] * u_ext[q];
  // right: j = n + q - NW <= i + NW, i.e. q <= i + 2 NW - n
  const int qend = min(2 * NW, i + 2 * NW - n + 1);
  for (int q = NW + threadIdx.x; q < qend; q += HL_BLOCK) acc += tab[n + q - NW - i + NW] * u_ext[q];
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) g[i] = acc;
}

// 2D exterior: tab[(k1 + NW)(2 NW + 1) + k2 + NW] is the coefficient of
// u(x_i + kh) in row i for |k|_inf <= NW, k != 0: W_k1 W_k2 nu(kh) with the
// row's kernel (tilted for an asymmetric measure), plus on the four nearest
// neighbours the local terms of their axis (diffusion, the u'' correction,
// the drift and an asymmetric measure's u' sum on the first axis).
__global__ void __launch_bounds__(HL_BLOCK) k_ext2_table(ProblemDev P, const double* cst, double* tab) {
  const int NW = P.n + 1, side = 2 * NW + 1;
  const long q = (long)blockIdx.x * HL_BLOCK + threadIdx.x;
  if (q >= (long)side * side) return;
  const int k1 = (int)(q / side) - NW, k2 = (int)(q % side) - NW;
  if (k1 == 0 && k2 == 0) {
    tab[q] = 0.0;
    return;
  }
  const double h = P.h;
  const double w = ((abs(k1) == NW) ? 0.5 * h : h) * ((abs(k2) == NW) ? 0.5 * h : h);
  const bool asym2 = P.kernel == HLEVY_KERNEL_TEMPERED_ASYM;
  double v = w * (asym2 ? nu_tilt2(P, k1, k2) : nu_at(P, h * sqrt((double)k1 * k1 + (double)k2 * k2)));
  if (abs(k1) + abs(k2) == 1) {
    const double beta = 0.5 * (cst[2] - cst[1]);
    const double beta_y = asym2 ? 0.5 * (cst[6] - cst[5]) : beta;
    if (k1 != 0) {
      const double b0 = asym2 ? P.b0 - cst[4] : P.b0;
      v += (beta + P.a) / (h * h) + (k1 > 0 ? 1.0 : -1.0) * b0 / (2.0 * h);
    } else {
      v += (beta_y + P.a) / (h * h) + (k2 > 0 ? 1.0 : -1.0) * P.b1 / (2.0 * h);
    }
  }
  tab[q] = v;
}
// g[p n + q] = sum over the exterior lattice points of the window of row
// (p, q) of tab u_ext; u_ext is an extended lattice, first coordinate
// slowest, lattice index a at position a + org per axis, ld per row.  One
// block per row, fixed-order sum.
__global__ void __launch_bounds__(HL_BLOCK) k_ext2_apply(const double* tab, const double* u_ext, int n, int ld,
                                                         int org, double* g) {
  __shared__ double red[4];
  const int NW = n + 1, side = 2 * NW + 1;
  const int p = blockIdx.x / n, q = blockIdx.x % n;
  double acc = 0.0;
  for (long e = threadIdx.x; e < (long)side * side; e += HL_BLOCK) {
    const int k1 = (int)(e / side) - NW, k2 = (int)(e % side) - NW;
    const int a1 = p + k1, a2 = q + k2;
    if (a1 >= 0 && a1 < n && a2 >= 0 && a2 < n) continue;   // interior point
    acc += tab[e] * u_ext[(size_t)(a1 + org) * ld + (a2 + org)];
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) g[blockIdx.x] = acc;
}

// 2D far field: tab[(k1 + next)(2 next + 1) + k2 + next] = (W_big - W_win)
// nu(kh), the product trapezoid weights of the square |k|_inf <= next (h/2 at
// |k_a| = next) less the window's (h/2 at |k_a| = NW), zero inside the
// window; the row's kernel (tilted for an asymmetric measure).
__global__ void __launch_bounds__(HL_BLOCK) k_far2_table(ProblemDev P, int next, double* tab) {
  const int NW = P.n + 1, side = 2 * next + 1;
  const long e = (long)blockIdx.x * HL_BLOCK + threadIdx.x;
  if (e >= (long)side * side) return;
  const int k1 = (int)(e / side) - next, k2 = (int)(e % side) - next;
  const double h = P.h;
  if (max(abs(k1), abs(k2)) < NW) {
    tab[e] = 0.0;
    return;
  }
  auto wb = [&](int k) { return abs(k) == next ? 0.5 * h : h; };
  auto ww = [&](int k) { return abs(k) == NW ? 0.5 * h : (abs(k) < NW ? h : 0.0); };
  const double w = wb(k1) * wb(k2) - ww(k1) * ww(k2);
  const double nu = P.kernel == HLEVY_KERNEL_TEMPERED_ASYM ? nu_tilt2(P, k1, k2)
                                                            : nu_at(P, h * sqrt((double)k1 * k1 + (double)k2 * k2));
  tab[e] = w * nu;
}
// out[0], out[1]: the measure of the region |y|_inf > R on the side y1 > 0,
// y1 < 0 (polar coordinates: four octants of 32 Gauss-Legendre nodes per
// side, the radial integral by the incomplete gamma function).  One block
// of 32 threads.
__global__ void k_far2_tails(ProblemDev P, double R, double* out) {
  __shared__ double glx[32], glw[32];
  gauss_legendre(32, threadIdx.x, &glx[threadIdx.x], &glw[threadIdx.x]);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double s = P.s, C = P.C;
  const bool tilt = P.kernel == HLEVY_KERNEL_TEMPERED_ASYM;
  const double lam0 = tilt ? 0.5 * (P.lam + P.lam_neg) : P.lam, th = tilt ? 0.5 * (P.lam_neg - P.lam) : 0.0;
  for (int side = 0; side < 2; ++side) {
    const double base = side == 0 ? -0.5 * M_PI : 0.5 * M_PI;
    double acc = 0.0;
    for (int oct = 0; oct < 4; ++oct)
      for (int q = 0; q < 32; ++q) {
        const double ph = base + 0.25 * M_PI * oct + 0.125 * M_PI * (glx[q] + 1.0), w = 0.125 * M_PI * glw[q];
        const double c = cos(ph), sn = sin(ph);
        const double r0 = R / fmax(fabs(c), fabs(sn));
        const double mu = lam0 - th * c;
        acc += w * (mu == 0.0 ? pow(r0, -2.0 * s) / (2.0 * s) : pow(mu, 2.0 * s) * upper_gamma(-2.0 * s, mu * r0));
      }
    out[side] = C * acc;
  }
}
// g[p n + q] += the far field of row (p, q): u_ext the extended lattice of
// indices -next .. n - 1 + next per axis; tails[0], tails[1] the measures of
// the two halves beyond the square.  One block per row, fixed-order sum.
__global__ void __launch_bounds__(HL_BLOCK) k_far2_apply(const double* tab, const double* tails, const double* u_ext,
                                                         int n, int next, double tail_left, double tail_right,
                                                         double* g) {
  __shared__ double red[4];
  const int NW = n + 1, side = 2 * next + 1, ld = n + 2 * next;
  const int p = blockIdx.x / n, q = blockIdx.x % n;
  double acc = 0.0;
  for (long e = threadIdx.x; e < (long)side * side; e += HL_BLOCK) {
    const int k1 = (int)(e / side) - next, k2 = (int)(e % side) - next;
    if (max(abs(k1), abs(k2)) < NW) continue;   // inside the window (interior values are not read)
    acc += tab[e] * u_ext[(size_t)(p + k1 + next) * ld + (q + k2 + next)];
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) g[blockIdx.x] += acc + tail_right * tails[0] + tail_left * tails[1];
}

// Far field f^{L_W} (eq. equ:fxy) of an exterior on an extended lattice, 1D.
// tab[2 (k - NW)] = W_k nu(kh), tab[2 (k - NW) + 1] = W_k nu(-kh) for
// k = NW .. next (W_k = h, h/2 at both ends), and after them the integrals
// of nu over y > next h and y < -next h.
__device__ double tail_of_nu(const ProblemDev& P, double rate, double R) {
  const double s = P.s;
  if (rate == 0.0) return P.C * pow(R, -2.0 * s) / (2.0 * s);
  return P.C * pow(rate, 2.0 * s) * upper_gamma(-2.0 * s, rate * R);
}
__global__ void __launch_bounds__(HL_BLOCK) k_far_table(ProblemDev P, int next, double* tab) {
  const int NW = P.n + 1, cnt = next - NW + 1;
  const int q = blockIdx.x * HL_BLOCK + threadIdx.x;
  const double h = P.h;
  if (q < cnt && next > NW) {
    const int k = NW + q;
    const double w = (k == NW || k == next) ? 0.5 * h : h;
    tab[2 * q] = w * nu_jump1(P, k);
    tab[2 * q + 1] = w * nu_jump1(P, -k);
  }
  if (q == 0) {
    const double R = next * h;
    const double rneg = P.kernel == HLEVY_KERNEL_TEMPERED_ASYM ? P.lam_neg : P.lam;
    tab[2 * cnt] = tail_of_nu(P, P.lam, R);
    tab[2 * cnt + 1] = tail_of_nu(P, rneg, R);
  }
}
// g[i] += the far field of row i: u_ext[0 .. next) are lattice indices
// -next .. -1, u_ext[next .. 2 next) indices n .. n + next - 1.  One block
// per row, fixed-order sum.
__global__ void __launch_bounds__(HL_BLOCK) k_far_apply(const double* tab, const double* u_ext, int n, int next,
                                                        double tail_left, double tail_right, double* g) {
  __shared__ double red[4];
  const int NW = n + 1, i = blockIdx.x, cnt = next - NW + 1;
  const double* left = u_ext;
  const double* right = u_ext + next;
  double acc = 0.0;
  if (next > NW)
    for (int q = threadIdx.x; q < cnt; q += HL_BLOCK) {
      const int k = NW + q;
      acc += tab[2 * q] * right[i + k - n] + tab[2 * q + 1] * left[i - k + next];
    }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) g[i] += acc + tail_right * tab[2 * cnt] + tail_left * tab[2 * cnt + 1];
}

// Fixed-rank Taylor factors of the Gaussian kernel (Sec. 3.3), one block per
// admissible leaf: with xbar the centre of the row cluster's bounding box,
// t0 = x_i - xbar and t = y_j - xbar per axis, column q holds
// U_iq = h^d C prod_ax (2 eps2)^n exp(-eps2 t0^2) t0^n / n! and
// V_jq = prod_ax exp(-eps2 t^2) t^n, the exponents n of term q taken in
// order of total degree (1D: n = q).  Coordinates are grid multiples
// (k + 1) h; the box origin cancels in the differences.  The rank is set to
// r (columns r.. of the capacity are left untouched).
__device__ __forceinline__ void taylor_exponents(int dim, int q, int& n1, int& n2) {
  if (dim == 1) {
    n1 = q;
    n2 = 0;
    return;
  }
  int deg = 0;
  while (q > deg) {
    q -= deg + 1;
    ++deg;
  }
  n2 = q;
  n1 = deg - q;
}
__device__ __forceinline__ double taylor_alpha(double e2, double t0, int n) {
  double v = exp(-e2 * t0 * t0);
  for (int k = 1; k <= n; ++k) v *= 2.0 * e2 * t0 / k;
  return v;
}
__device__ __forceinline__ double taylor_beta(double e2, double t, int n) {
  double v = exp(-e2 * t * t);
  for (int k = 1; k <= n; ++k) v *= t;
  return v;
}
__global__ void __launch_bounds__(HL_BLOCK) k_taylor(ProblemDev P, const int32_t* perm, const LeafDesc* L,
                                                     const int32_t* ids, int32_t* rank, int r) {
  __shared__ double red[4];
  __shared__ double cen[2];
  const int leaf = ids[blockIdx.x];
  const LeafDesc d = L[leaf];
  const double h = P.h;
  // bounding box of the row cluster, per axis
  for (int ax = 0; ax < P.dim; ++ax) {
    double mn = 1e300, mx = -1e300;
    for (int i = threadIdx.x; i < d.m; i += HL_BLOCK) {
      const int pi = perm[d.rlo + i];
      const int g = P.dim == 1 ? pi : (ax == 0 ? pi / P.n : pi % P.n);
      const double x = (g + 1) * h;
      mn = fmin(mn, x);
      mx = fmax(mx, x);
    }
    const double lo = -block_max(-mn, red);
    const double hi = block_max(mx, red);
    if (threadIdx.x == 0) cen[ax] = 0.5 * (lo + hi);
    __syncthreads();
  }
  const double scale = (P.dim == 1 ? h : h * h) * P.C;
  const double e2 = P.eps2;
  for (int e = threadIdx.x; e < d.m * r; e += HL_BLOCK) {
    const int i = e % d.m, q = e / d.m;
    int n1, n2;
    taylor_exponents(P.dim, q, n1, n2);
    const int pi = perm[d.rlo + i];
    double v;
    if (P.dim == 1) {
      v = taylor_alpha(e2, (pi + 1) * h - cen[0], n1);
    } else {
      v = taylor_alpha(e2, (pi / P.n + 1) * h - cen[0], n1) * taylor_alpha(e2, (pi % P.n + 1) * h - cen[1], n2);
    }
    d.A[i + (size_t)d.m * q] = scale * v;
  }
  for (int e = threadIdx.x; e < d.n * r; e += HL_BLOCK) {
    const int j = e % d.n, q = e / d.n;
    int n1, n2;
    taylor_exponents(P.dim, q, n1, n2);
    const int pj = perm[d.clo + j];
    double v;
    if (P.dim == 1) {
      v = taylor_beta(e2, (pj + 1) * h - cen[0], n1);
    } else {
      v = taylor_beta(e2, (pj / P.n + 1) * h - cen[0], n1) * taylor_beta(e2, (pj % P.n + 1) * h - cen[1], n2);
    }
    d.B[j + (size_t)d.n * q] = v;
  }
  if (threadIdx.x == 0) rank[leaf] = r;
}

// one block per dense leaf: fill G entries (col-major)
__global__ void __launch_bounds__(HL_BLOCK) k_fill_dense(ProblemDev P, const double* cst,
                                                         const int32_t* perm,
                                                         const LeafDesc* L, const int32_t* ids) {
  const LeafDesc d = L[ids[blockIdx.x]];
  const int tot = d.m * d.n;
  for (int e = threadIdx.x; e < tot; e += blockDim.x) {
    int i = e % d.m, j = e / d.m;
    d.A[e] = gen_entry(P, cst, perm, d.rlo + i, d.clo + j);
  }
}

// Partially pivoted ACA of an admissible block, one block per leaf.
// Writes U (m x kcap), V (n x kcap) and the rank.  Stopping rule:
// ||u_k|| ||v_k|| <= eps ||S_k||_F with the running Frobenius estimate.
// First pivot row is row 0; the next pivot row maximises |u_k| over unused
// rows (ties: lowest index); the pivot column maximises the residual row.
__global__ void __launch_bounds__(HL_BLOCK) k_aca(ProblemDev P, const int32_t* perm,
                                                  const LeafDesc* L, const int32_t* ids,
                                                  double* Ubuf, double* Vbuf, const int64_t* uoff,
                                                  const int64_t* voff, int32_t* ranks, int kcap,
                                                  double eps) {
  __shared__ double red[4];
  __shared__ double rv[4];
  __shared__ int ri[4];
  __shared__ double coef[KMAX];
  __shared__ double dots[2 * KMAX];
  __shared__ uint32_t used[LR_ROWS_MAX / 32];   // one bit per row of the block
  const LeafDesc d = L[ids[blockIdx.x]];
  double* U = Ubuf + uoff[blockIdx.x];
  double* V = Vbuf + voff[blockIdx.x];
  const int m = d.m, n = d.n;
  const int kmax = min(kcap, min(m, n));
  for (int q = threadIdx.x; q < LR_ROWS_MAX / 32; q += blockDim.x) used[q] = 0u;
  __syncthreads();
  int i = 0, k = 0;
  double normS2 = 0.0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  while (k < kmax) {
    // residual row i -> V[:, k]
    for (int q = threadIdx.x; q < k; q += blockDim.x) coef[q] = U[i + (size_t)m * q];
    __syncthreads();
    double best = -1.0;
    int bidx = 0x7fffffff;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      double v = far_entry(P, perm, d.rlo + i, d.clo + j);
      for (int q = 0; q < k; ++q) v -= coef[q] * V[j + (size_t)n * q];
      V[j + (size_t)n * k] = v;
      double a = fabs(v);
      if (a > best || (a == best && j < bidx)) { best = a; bidx = j; }
    }
    // argmax over the block (ties -> lowest index)
    for (int o = 32; o > 0; o >>= 1) {
      double ob = __shfl_xor(best, o, 64);
      int oi = __shfl_xor(bidx, o, 64);
      if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
    }
    if (lane == 0) { rv[w] = best; ri[w] = bidx; }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < 4; ++q)
        if (rv[q] > rv[0] || (rv[q] == rv[0] && ri[q] < ri[0])) { rv[0] = rv[q]; ri[0] = ri[q]; }
    }
    __syncthreads();
    const int jp = ri[0];
    const double delta = V[jp + (size_t)n * k];
    __syncthreads();
    if (!(fabs(delta) > 0.0)) break;
    const double inv = 1.0 / delta;
    for (int j = threadIdx.x; j < n; j += blockDim.x) V[j + (size_t)n * k] *= inv;
    for (int q = threadIdx.x; q < k; q += blockDim.x) coef[q] = V[jp + (size_t)n * q];
    __syncthreads();
    // residual column jp -> U[:, k]
    for (int r = threadIdx.x; r < m; r += blockDim.x) {
      double v = far_entry(P, perm, d.rlo + r, d.clo + jp);
      for (int q = 0; q < k; ++q) v -= coef[q] * U[r + (size_t)m * q];
      U[r + (size_t)m * k] = v;
    }
    __syncthreads();
    // norms and cross terms with earlier pairs
    for (int q = 0; q <= k; ++q) {
      double pu = 0.0, pv = 0.0;
      for (int r = threadIdx.x; r < m; r += blockDim.x) pu += U[r + (size_t)m * q] * U[r + (size_t)m * k];
      for (int j = threadIdx.x; j < n; j += blockDim.x) pv += V[j + (size_t)n * q] * V[j + (size_t)n * k];
      pu = block_sum(pu, red);
      pv = block_sum(pv, red);
      if (threadIdx.x == 0) { dots[q] = pu; dots[KMAX + q] = pv; }
    }
    __syncthreads();
    double nu2 = dots[k], nv2 = dots[KMAX + k];
    double cross = 0.0;
    for (int q = 0; q < k; ++q) cross += dots[q] * dots[KMAX + q];
    normS2 += nu2 * nv2 + 2.0 * cross;
    if (threadIdx.x == 0) used[i >> 5] |= 1u << (i & 31);
    __syncthreads();
    ++k;
    if (sqrt(nu2 * nv2) <= eps * sqrt(fmax(normS2, 0.0))) break;
    // next pivot row: argmax |U[:, k-1]| over unused rows
    best = -1.0;
    bidx = 0x7fffffff;
    for (int r = threadIdx.x; r < m; r += blockDim.x) {
      if (used[r >> 5] & (1u << (r & 31))) continue;
      double a = fabs(U[r + (size_t)m * (k - 1)]);
      if (a > best || (a == best && r < bidx)) { best = a; bidx = r; }
    }
    for (int o = 32; o > 0; o >>= 1) {
      double ob = __shfl_xor(best, o, 64);
      int oi = __shfl_xor(bidx, o, 64);
      if (ob > best || (ob == best && oi < bidx)) { best = ob; bidx = oi; }
    }
    if (lane == 0) { rv[w] = best; ri[w] = bidx; }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int q = 1; q < 4; ++q)
        if (rv[q] > rv[0] || (rv[q] == rv[0] && ri[q] < ri[0])) { rv[0] = rv[q]; ri[0] = ri[q]; }
    }
    __syncthreads();
    if (rv[0] < 0.0) break;   // every row used
    i = ri[0];
    __syncthreads();
  }
  if (threadIdx.x == 0) ranks[blockIdx.x] = k;
}

// ---------------------------------------------------------------------------
// rounded addition: Gram (double-double) -> pivoted Cholesky -> Jacobi SVD
// ---------------------------------------------------------------------------
constexpr int RA_YS = 32;   // row stride of Y_U / Y_V (>= every rank capacity)

// columns of a low-rank term (its rank, or its share of a split term)
__device__ __forceinline__ int term_rank(const Term& tm) {
  const int k = tm.k ? *tm.k : tm.kfix;
  return tm.klim > 0 ? min(max(k - tm.kofs, 0), tm.klim) : k;
}

struct ColMap {
  int K, kC, nt, tb;   // tb: first term of this concatenation (relative to T.tbeg)
  int off[KMAX + 1];
  int kt[KMAX];
};

// The next concatenation of a target's term list: the target's kC columns
// and terms [t0, t0 + nt), nt as large as the width limit allows (at least
// one term, at most 64).  Run by the 64 lanes of the first wavefront: each
// lane reads one term's rank, a shuffle prefix sum gives the column
// offsets, and the terms that fit form a run from lane 0.
__device__ void build_colmap_chunk(const LFlushTarget& T, const Term* terms, int kC, int t0, int limit, ColMap& cm) {
  const int lane = threadIdx.x & 63;
  const int avail = min(64, T.tcount - t0);
  const int kt = lane < avail ? term_rank(terms[T.tbeg + t0 + lane]) : 0;
  int incl = kt;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(incl, o, 64);
    if (lane >= o) incl += v;
  }
  const bool take = lane < avail && (lane == 0 || kC + incl <= limit);
  const int nt = __popcll(__ballot(take));
  if (take) {
    cm.off[lane] = kC + incl - kt;
    cm.kt[lane] = kt;
  }
  if (lane == nt - 1) {
    cm.off[nt] = kC + incl;
    cm.K = kC + incl;
  }
  if (lane == 0) {
    cm.kC = kC;
    cm.tb = t0;
    cm.nt = nt;
  }
}

// the whole term list of one rounded addition (at most 64 terms: every
// term has at least one column and a concatenation at most KMAX)
__device__ void build_colmap(const LFlushTarget& T, const Term* terms, int kC, ColMap& cm) {
  build_colmap_chunk(T, terms, kC, 0, 1 << 30, cm);
}

// value of column j of the concatenated factor on side 0 (U side) or 1 (V side)
__device__ __forceinline__ double side_val(const LFlushTarget& T, const Term* terms, const ColMap& cm,
                                           int side, int row, int j) {
  if (j < cm.kC) return side == 0 ? T.U[row + (size_t)T.m * j] : T.V[row + (size_t)T.n * j];
  int t = 0;
  while (j >= cm.off[t + 1]) ++t;
  const Term& tm = terms[T.tbeg + cm.tb + t];
  int c = j - cm.off[t];
  if (side == 0) {
    int rr = row - tm.ro;
    if (rr < 0 || rr >= tm.mr) return 0.0;
    return tm.sign * tm.U[rr + (size_t)tm.ldu * c];
  }
  int rr = row - tm.co;
  if (rr < 0 || rr >= tm.nc) return 0.0;
  return tm.W[rr + (size_t)tm.ldw * c];
}

__device__ __forceinline__ int pair_index(int p, int q) { return q * (q + 1) / 2 + p; }  // p <= q
__host__ __device__ inline int npairs(int K) { return K * (K + 1) / 2; }


// Pivoted Cholesky (double-double) of the Gram G (K x K, stride ks, in
// Gh/Gl), one block of 256 threads, every step parallel.  Writes R (rank x K,
// original column order, row stride ks) and returns the rank; columns whose
// remaining diagonal falls below 1e-32 of the largest initial diagonal are
// dropped.  Pivot = largest remaining diagonal (ties: lowest index).
__device__ int pivoted_cholesky(double* Gh, double* Gl, double* R, int K, int ks, int* sel, double* rowh,
                                double* rowl, int* sint, double cut2, bool use_dd) {
  const int tid = threadIdx.x, lane = tid & 63;
  for (int e = tid; e < ks * ks; e += HL_BLOCK) R[e] = 0.0;
  if (tid < KMAX) sel[tid] = 0;
  __syncthreads();
  double dmax0 = 0.0;
  if (tid < 64) {
    double v = lane < K ? Gh[lane * ks + lane] : 0.0;
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    dmax0 = v;
  }
  __shared__ double s_dmax0;
  if (tid == 0) s_dmax0 = dmax0;
  __syncthreads();
  dmax0 = s_dmax0;
  int r = 0;
  for (int j = 0; j < K; ++j) {
    if (tid < 64) {
      // argmax of the remaining diagonal over the first wavefront
      double vh = -1.0, vl = 0.0;
      int idx = 0x7fffffff;
      if (lane < K && !sel[lane]) { vh = Gh[lane * ks + lane]; vl = use_dd ? Gl[lane * ks + lane] : 0.0; idx = lane; }
      for (int o = 32; o > 0; o >>= 1) {
        double oh = __shfl_xor(vh, o, 64), ol = __shfl_xor(vl, o, 64);
        int oi = __shfl_xor(idx, o, 64);
        if (oh > vh || (oh == vh && (ol > vl || (ol == vl && oi < idx)))) { vh = oh; vl = ol; idx = oi; }
      }
      if (tid == 0) {
        int best = (idx < K && vh > cut2 * dmax0 && vh > 0.0) ? idx : -1;
        sint[0] = best;
        if (best >= 0) sel[best] = 1;
      }
    }
    __syncthreads();
    const int p = sint[0];
    if (p < 0) break;
    const dd gpp = {Gh[p * ks + p], use_dd ? Gl[p * ks + p] : 0.0};
    const dd rjj = use_dd ? dd_sqrt(gpp) : dd{sqrt(gpp.hi), 0.0};
    const dd rinv = use_dd ? dd_div({1.0, 0.0}, rjj) : dd{1.0 / rjj.hi, 0.0};
    for (int q = tid; q < K; q += HL_BLOCK) {
      dd v;
      const int a = min(p, q), b = max(p, q);   // upper triangle holds G
      if (q == p) v = rjj;
      else if (sel[q]) v = {0.0, 0.0};
      else if (use_dd) v = dd_mul({Gh[a * ks + b], Gl[a * ks + b]}, rinv);
      else v = {Gh[a * ks + b] * rinv.hi, 0.0};
      rowh[q] = v.hi;
      rowl[q] = v.lo;
      R[j * ks + q] = v.hi + v.lo;
    }
    __syncthreads();
    // Schur complement update of the upper triangle (q1 <= q2), 16 x 16
    // thread grid; the lower triangle is read through the symmetry
    for (int q1 = tid >> 4; q1 < K; q1 += 16) {
      if (sel[q1]) continue;
      const dd a = {rowh[q1], rowl[q1]};
      for (int q2 = q1 + (tid & 15); q2 < K; q2 += 16) {
        if (sel[q2]) continue;
        if (use_dd) {
          dd gv = {Gh[q1 * ks + q2], Gl[q1 * ks + q2]};
          gv = dd_add(gv, dd_neg(dd_mul(a, {rowh[q2], rowl[q2]})));
          Gh[q1 * ks + q2] = gv.hi;
          Gl[q1 * ks + q2] = gv.lo;
        } else {
          Gh[q1 * ks + q2] -= a.hi * rowh[q2];
        }
      }
    }
    __syncthreads();
    r = j + 1;
  }
  __syncthreads();
  return r;
}

// One block per target: Gram sums -> R_A, R_B (pivoted Cholesky in
// double-double) -> M = R_A R_B^T -> one-sided Jacobi SVD -> truncation at
// the relative Frobenius tolerance -> Y_U = R_B^T Z_r and
// Y_V = R_A^T W_r Sigma_r^{-1}, so that U_new = A Y_U and V_new = B Y_V.
// Dynamic LDS: 4 ks^2 doubles, ks >= the widest concatenation of the launch.
__global__ void __launch_bounds__(HL_BLOCK) k_flush_core(const LFlushTarget* tg, const Term* terms, double tol,
                                                         int ks) {
  extern __shared__ double smem[];
  const int ld = ks + 1;   // odd column stride for M and Z: no bank conflicts between pairs
  double* Gh = smem;
  double* Gl = Gh + ks * ld;
  double* RA = Gl + ks * ld;
  double* RB = RA + ks * ks;
  __shared__ ColMap cm;
  __shared__ int sel[KMAX];
  __shared__ double rowh[KMAX], rowl[KMAX];
  __shared__ int sint[4];
  __shared__ double sig[KMAX];
  __shared__ int order[KMAX];
  __shared__ int rot_count;
  const LFlushTarget T = tg[blockIdx.x];
  const int tid = threadIdx.x;
  const int kC = T.rank ? *T.rank : 0;
  if (tid < 64) build_colmap(T, terms, kC, cm);
  __syncthreads();
  const int K = cm.K;
  const int Kc = T.Kcap;
  const int np = npairs(Kc);
  int rk[2];
  for (int side = 0; side < 2; ++side) {
    const int nch = side == 0 ? T.nchA : T.nchB;
    const double* src = T.ws + (size_t)(side == 0 ? 0 : T.nchA) * np * 2;
    const int npk = npairs(K);
    for (int idx = tid; idx < npk; idx += HL_BLOCK) {
      int q = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
      while (q * (q + 1) / 2 > idx) --q;
      while ((q + 1) * (q + 2) / 2 <= idx) ++q;
      const int p = idx - q * (q + 1) / 2;
      dd s = {src[2 * idx], src[2 * idx + 1]};
      for (int c = 1; c < nch; c += 4) {
        double h[4], l[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          h[u] = 0.0;
          l[u] = 0.0;
          if (c + u < nch) {
            h[u] = src[(size_t)(c + u) * np * 2 + 2 * idx];
            l[u] = src[(size_t)(c + u) * np * 2 + 2 * idx + 1];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) s = dd_add(s, {h[u], l[u]});
      }
      Gh[p * ks + q] = s.hi;
      Gl[p * ks + q] = s.lo;
      Gh[q * ks + p] = s.hi;
      Gl[q * ks + p] = s.lo;
    }
    __syncthreads();
    // directions of a factor below 1e-2 tol of its largest column cannot
    // change the truncated product beyond the tolerance: stop there
    const double cut = fmax(1e-16, 1e-2 * tol);
    // double-double only where the tolerance needs digits below sqrt(eps)
    rk[side] = pivoted_cholesky(Gh, Gl, side == 0 ? RA : RB, K, ks, sel, rowh, rowl, sint,
                                fmax(cut * cut, 1e-32), radd_dd(tol));
  }
  const int rA = rk[0], rB = rk[1];
  // M (rA x rB) and Z (rB x rB), column-major with stride ld
  double* M = Gh;
  double* Z = Gl;
  for (int e = tid; e < ks * ld; e += HL_BLOCK) { M[e] = 0.0; Z[e] = 0.0; }
  __syncthreads();
  for (int e = tid; e < rA * rB; e += HL_BLOCK) {
    int i = e % rA, j = e / rA;
    double s = 0.0;
    for (int q = 0; q < K; ++q) s += RA[i * ks + q] * RB[j * ks + q];
    M[i + ld * j] = s;
  }
  for (int e = tid; e < rB; e += HL_BLOCK) Z[e + ld * e] = 1.0;
  __syncthreads();
  // one-sided Jacobi on the columns of M, disjoint pairs per round
  const int nn = rB + (rB & 1);
  const int g = tid >> 3, l8 = tid & 7;
  for (int sweep = 0; sweep < 40 && nn >= 2; ++sweep) {
    if (tid == 0) rot_count = 0;
    __syncthreads();
    for (int rd = 0; rd < nn - 1; ++rd) {
      if (g < nn / 2) {
        int a = (rd + g) % (nn - 1);
        int b = (g == 0) ? nn - 1 : (rd - g + nn - 1) % (nn - 1);
        if (a > b) { int tt = a; a = b; b = tt; }
        const bool active = (b < rB);
        double al = 0.0, be = 0.0, ga = 0.0;
        if (active) {
          for (int i = l8; i < rA; i += 8) {
            double x = M[i + ld * a], y = M[i + ld * b];
            al += x * x; be += y * y; ga += x * y;
          }
        }
        for (int o = 4; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, 8);
          be += __shfl_xor(be, o, 8);
          ga += __shfl_xor(ga, o, 8);
        }
        // rotate while the pair is not orthogonal to working accuracy
        if (active && ga != 0.0 && fabs(ga) > 4e-15 * sqrt(al * be)) {
          double zeta = (be - al) / (2.0 * ga);
          double tq = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double c = 1.0 / sqrt(1.0 + tq * tq), s = c * tq;
          for (int i = l8; i < rA; i += 8) {
            double x = M[i + ld * a], y = M[i + ld * b];
            M[i + ld * a] = c * x - s * y;
            M[i + ld * b] = s * x + c * y;
          }
          for (int i = l8; i < rB; i += 8) {
            double x = Z[i + ld * a], y = Z[i + ld * b];
            Z[i + ld * a] = c * x - s * y;
            Z[i + ld * b] = s * x + c * y;
          }
          if (l8 == 0) atomicAdd(&rot_count, 1);
        }
      }
      __syncthreads();
    }
    const int rc = rot_count;
    __syncthreads();
    if (rc == 0) break;
  }
  for (int c = tid; c < rB; c += HL_BLOCK) {
    double s = 0.0;
    for (int i = 0; i < rA; ++i) s += M[i + ld * c] * M[i + ld * c];
    sig[c] = sqrt(s);
  }
  __syncthreads();
  // rank-based sort (descending, ties by index) and truncation via a suffix
  // sum of squared singular values, both in the first wavefront
  if (tid < 64) {
    const int c = tid;
    double sc = c < rB ? sig[c] : -1.0;
    if (c < rB) {
      int pos = 0;
      for (int c2 = 0; c2 < rB; ++c2) {
        double s2 = sig[c2];
        pos += (s2 > sc || (s2 == sc && c2 < c)) ? 1 : 0;
      }
      order[pos] = c;
    }
  }
  __syncthreads();
  if (tid < 64) {
    const int lane = tid;
    double v = lane < rB ? sig[order[lane]] : 0.0;
    double sq = v * v;
    // suffix sum: suf[lane] = sum_{c >= lane} sq[c]
    double suf = sq;
    for (int o = 1; o < 64; o <<= 1) {
      double w = __shfl_down(suf, o, 64);
      if (lane + o < 64) suf += w;
    }
    double tot = __shfl(suf, 0, 64);
    // keep column c unless the tail starting at c fits within tol^2 * tot
    int keep = (lane < rB && suf > tol * tol * tot) ? 1 : 0;
    for (int o = 32; o > 0; o >>= 1) keep += __shfl_xor(keep, o, 64);
    if (lane == 0) {
      int r = (tot > 0.0) ? keep : 0;
      int ovf = 0;
      if (r > T.kcap) { r = T.kcap; ovf = 1; }
      sint[0] = r;
      T.info[0] = kC;
      T.info[1] = r;
      T.info[2] = ovf;
      if (ovf && T.overflow) atomicAdd(T.overflow, 1);
      if (T.rank) *T.rank = r;
    }
  }
  __syncthreads();
  const int r = sint[0];
  // Y_U, Y_V: K x RA_YS each, row q at q * RA_YS, zero beyond r (k_flush_expand)
  double* YU = T.ws + (size_t)(T.nchA + T.nchB) * np * 2;
  double* YV = YU + (size_t)K * RA_YS;
  for (int e = tid; e < K * RA_YS; e += HL_BLOCK) {
    const int q = e / RA_YS, c = e % RA_YS;
    double su = 0.0, sv = 0.0;
    if (c < r) {
      const int oc = order[c];
      for (int i = 0; i < rB; ++i) su += RB[i * ks + q] * Z[i + ld * oc];
      for (int i = 0; i < rA; ++i) sv += RA[i * ks + q] * M[i + ld * oc];
      const double sg = sig[oc];
      sv /= sg * sg;
    }
    YU[e] = su;
    YV[e] = sv;
  }
}

// Fast rounded addition for concatenations of at most 48 columns.
//
// With A (m x K) and B (n x K) the concatenated factors of C = A B^T,
// G_A = A^T A, G_B = B^T B (double-double):
//  1. pivoted Cholesky G_B = R_B^T R_B  (B = Q_B R_B, rank rB)
//  2. T1 = G_A R_B^T (K x rB) and G_M = R_B T1 = M^T M for M = R_A R_B^T
//  3. pivoted Cholesky of G_M, stopped as soon as the trace of the
//     remaining Schur complement (= ||M - M_J T||_F^2, the squared error of
//     the column-subset approximation) is <= tol^2 trace(G_M) or the rank
//     capacity is reached: pivots J, upper factor R_MJ (r x r)
//  4. U_new = A Y_U, Y_U = R_B[J,:]^T R_MJ^{-1}  (orthonormal columns: Q_A M_J R_MJ^{-1})
//     V_new = B Y_V, Y_V = T1[:, J] R_MJ^{-1}    (= C^T U_new)
// so C - U_new V_new^T = (I - P) C with P the projector on span(U_new) and
// ||C - U_new V_new^T||_F = ||M - M_J T||_F <= tol ||C||_F.
// Schur complements are stored in their upper triangle; row j of each
// Cholesky factor is written into the storage row of its pivot.
// One barrier per step: every wavefront selects the pivot itself from the
// remaining diagonal (largest, ties to the lowest index; identical in all
// wavefronts: a DPP max-reduction and a ballot), the selected set is a register bit mask, and the factor row
// of step j is written into its storage row p_j during step j + 1, when no
// thread reads row p_j any more (reads and the Schur update touch only
// unselected rows and columns).  Row p_j then holds rjj at p_j, 0 at the
// columns selected before p_j and S[p_j, q] / rjj elsewhere.  Stops after
// rmax steps, at a non-positive pivot, or when
//   mode 0: the largest remaining diagonal <= thr * (initial largest),
//   mode 1: the remaining trace <= thr * (initial trace).
// piv[j] = pivot of step j; *ref_out = the initial reference.  Returns the
// rank (the same value in every thread).
__device__ __forceinline__ void pchol_row(double* Sh, double* Sl, int K, int ls, int p, unsigned long long before,
                                          dd rjj, dd rinv, bool use_dd) {
  for (int q = threadIdx.x; q < K; q += HL_BLOCK) {
    dd v;
    if (q == p) {
      v = rjj;
    } else if ((before >> q) & 1ull) {
      v = {0.0, 0.0};
    } else {
      const int a = min(p, q), b = max(p, q);
      v = use_dd ? dd_mul({Sh[a * ls + b], Sl[a * ls + b]}, rinv) : dd{Sh[a * ls + b] * rinv.hi, 0.0};
    }
    Sh[p * ls + q] = v.hi;
    if (use_dd) Sl[p * ls + q] = v.lo;
  }
}

// Wavefront reductions with DPP moves inside each 16-lane row (quad
// permutations, then row rotations by 4 and 8) and readlane across the four
// rows; every lane gets the same value, computed in the same order in every
// wavefront.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double rdlane_d(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double wave_max_dpp(double v) {
  v = fmax(v, dpp_d<0xB1>(v));    // quad_perm 1,0,3,2
  v = fmax(v, dpp_d<0x4E>(v));    // quad_perm 2,3,0,1
  v = fmax(v, dpp_d<0x124>(v));   // row_ror 4
  v = fmax(v, dpp_d<0x128>(v));   // row_ror 8: every lane holds its row maximum
  return fmax(fmax(rdlane_d(v, 0), rdlane_d(v, 16)), fmax(rdlane_d(v, 32), rdlane_d(v, 48)));
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x124>(v);
  v += dpp_d<0x128>(v);   // lane 16 i holds the sum of row i
  return (rdlane_d(v, 0) + rdlane_d(v, 16)) + (rdlane_d(v, 32) + rdlane_d(v, 48));
}

__device__ int pchol_inplace(double* Sh, double* Sl, int K, int ls, int* piv, double* ref_out, int mode,
                             double thr, int rmax, bool use_dd) {
  const int tid = threadIdx.x, lane = tid & 63;
  double ref;
  {
    const double d = lane < K ? Sh[lane * ls + lane] : 0.0;
    ref = mode == 0 ? wave_max_dpp(d) : wave_sum_dpp(d);
  }
  if (tid == 0) *ref_out = ref;
  unsigned long long selm = 0ull;
  int r = 0, pprev = -1;
  dd rjj_prev{0.0, 0.0}, rinv_prev{0.0, 0.0};
  for (int j = 0; j < K && j < rmax; ++j) {
    if (pprev >= 0) {
      pchol_row(Sh, Sl, K, ls, pprev, selm & ~(1ull << pprev), rjj_prev, rinv_prev, use_dd);
      pprev = -1;
    }
    // pivot: the largest remaining diagonal (double-double: then the
    // largest low part), ties to the lowest index
    const bool un = lane < K && !((selm >> lane) & 1ull);
    const double vh = un ? Sh[lane * ls + lane] : -1.0;
    const double mx = wave_max_dpp(vh);
    unsigned long long cand = __ballot(un && vh == mx);
    if (use_dd) {
      const double vl = un ? Sl[lane * ls + lane] : 0.0;
      const double ml = wave_max_dpp(((cand >> lane) & 1ull) ? vl : -INFINITY);
      cand &= __ballot(vl == ml);
    }
    const double tr = mode == 1 ? wave_sum_dpp(un ? vh : 0.0) : 0.0;
    bool stop = cand == 0ull || !(mx > 0.0);
    stop = stop || (mode == 0 ? !(mx > thr * ref) : !(tr > thr * ref));
    if (stop) break;
    const int p = __ffsll((long long)cand) - 1;
    if (tid == 0) piv[j] = p;
    selm |= 1ull << p;
    const dd gpp = {Sh[p * ls + p], use_dd ? Sl[p * ls + p] : 0.0};
    const dd rjj = use_dd ? dd_sqrt(gpp) : dd{sqrt(gpp.hi), 0.0};
    const dd rinv = use_dd ? dd_div({1.0, 0.0}, rjj) : dd{1.0 / rjj.hi, 0.0};
    // Schur complement of the unselected rows and columns (upper triangle)
    for (int q1 = tid >> 4; q1 < K; q1 += HL_BLOCK / 16) {
      if ((selm >> q1) & 1ull) continue;
      const int a1 = min(p, q1), b1 = max(p, q1);
      const dd x1 = use_dd ? dd_mul({Sh[a1 * ls + b1], Sl[a1 * ls + b1]}, rinv) : dd{Sh[a1 * ls + b1] * rinv.hi, 0.0};
      for (int q2 = q1 + (tid & 15); q2 < K; q2 += 16) {
        if ((selm >> q2) & 1ull) continue;
        const int a2 = min(p, q2), b2 = max(p, q2);
        if (use_dd) {
          const dd x2 = dd_mul({Sh[a2 * ls + b2], Sl[a2 * ls + b2]}, rinv);
          dd gv = {Sh[q1 * ls + q2], Sl[q1 * ls + q2]};
          gv = dd_add(gv, dd_neg(dd_mul(x1, x2)));
          Sh[q1 * ls + q2] = gv.hi;
          Sl[q1 * ls + q2] = gv.lo;
        } else {
          Sh[q1 * ls + q2] -= x1.hi * (Sh[a2 * ls + b2] * rinv.hi);
        }
      }
    }
    __syncthreads();
    pprev = p;
    rjj_prev = rjj;
    rinv_prev = rinv;
    r = j + 1;
  }
  if (pprev >= 0) pchol_row(Sh, Sl, K, ls, pprev, selm & ~(1ull << pprev), rjj_prev, rinv_prev, use_dd);
  __syncthreads();
  return r;
}

// Steps 1-4 of the fast rounded addition on the Gram matrices G_A (in Y) and
// G_B (in X), all with row stride ks (odd: no LDS bank conflicts between
// rows); Y_U and Y_V (K x r, row q at q * RA_YS, zero beyond r) go to LDS.
// Writes the target's info / rank and returns r.
__device__ int radd_core(const LFlushTarget& T, int kC, int K, double tol, int ks, double* Xh, double* Xl,
                         double* Yh, double* Yl, double* Zh, double* Zl, double* YU, double* YV, int* pivB,
                         int* pivM, double* sref, bool b_orth = false) {
  const int tid = threadIdx.x;
  const bool use_dd = radd_dd(tol);
  // 1. G_B = R_B^T R_B; directions below 1e-2 tol of the largest are dropped
  const double cut = fmax(1e-16, 1e-2 * tol);
  int rB;
  if (b_orth) {
    // G_B = I (G_B is not formed): the pivoted Cholesky of the identity
    // selects 0, 1, .. K-1 and leaves R_B = I, so T1 = G_M = G_A
    for (int e = tid; e < K * K; e += HL_BLOCK) {
      const int q = e / K, p = e - q * K;
      Xh[q * ks + p] = q == p ? 1.0 : 0.0;
      Zh[q * ks + p] = Yh[q * ks + p];
      if (use_dd) {
        Xl[q * ks + p] = 0.0;
        Zl[q * ks + p] = Yl[q * ks + p];
      }
    }
    for (int j = tid; j < K; j += HL_BLOCK) pivB[j] = j;
    if (tid == 0) sref[0] = 1.0;
    __syncthreads();
    rB = K;
  } else {
    rB = pchol_inplace(Xh, Xl, K, ks, pivB, sref, 0, fmax(cut * cut, 1e-32), KMAX, use_dd);
  }
  // 2. T1[q][j] = sum_p G_A[q][p] R_B[j][p]
  for (int e = tid; e < K * rB && !b_orth; e += HL_BLOCK) {
    const int q = e / rB, j = e - q * rB;
    const double* rb_h = Xh + pivB[j] * ks;
    const double* rb_l = Xl + pivB[j] * ks;
    dd s = {0.0, 0.0};
    if (use_dd) {
      for (int p = 0; p < K; ++p) s = dd_add(s, dd_mul({Yh[q * ks + p], Yl[q * ks + p]}, {rb_h[p], rb_l[p]}));
    } else {
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      int p = 0;
      for (; p + 4 <= K; p += 4)
#pragma unroll
        for (int u = 0; u < 4; ++u) s4[u] += Yh[q * ks + p + u] * rb_h[p + u];
      for (; p < K; ++p) s4[0] += Yh[q * ks + p] * rb_h[p];
      s.hi = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
    Zh[q * ks + j] = s.hi;
    if (use_dd) Zl[q * ks + j] = s.lo;
  }
  __syncthreads();
  // G_M[i][j] = sum_p R_B[i][p] T1[p][j]  (overwrites G_A)
  for (int e = tid; e < rB * rB && !b_orth; e += HL_BLOCK) {
    const int i = e / rB, j = e - i * rB;
    const double* rb_h = Xh + pivB[i] * ks;
    const double* rb_l = Xl + pivB[i] * ks;
    dd s = {0.0, 0.0};
    if (use_dd) {
      for (int p = 0; p < K; ++p) s = dd_add(s, dd_mul({rb_h[p], rb_l[p]}, {Zh[p * ks + j], Zl[p * ks + j]}));
    } else {
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      int p = 0;
      for (; p + 4 <= K; p += 4)
#pragma unroll
        for (int u = 0; u < 4; ++u) s4[u] += rb_h[p + u] * Zh[(p + u) * ks + j];
      for (; p < K; ++p) s4[0] += rb_h[p] * Zh[p * ks + j];
      s.hi = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
    Yh[i * ks + j] = s.hi;
    if (use_dd) Yl[i * ks + j] = s.lo;
  }
  __syncthreads();
  // 3. rank-revealing Cholesky of G_M with the truncation tolerance
  const int r = pchol_inplace(Yh, Yl, rB, ks, pivM, sref + 1, 1, tol * tol, T.kcap, use_dd);
  if (tid == 0) {
    int ovf = 0;
    if (r == T.kcap && r < rB) {
      // capacity reached: flag it if the remaining trace still exceeds the tolerance
      unsigned long long sel = 0ull;
      for (int c = 0; c < r; ++c) sel |= 1ull << pivM[c];
      double tr = 0.0;
      for (int q = 0; q < rB; ++q)
        if (!((sel >> q) & 1ull)) tr += Yh[q * ks + q];
      ovf = tr > tol * tol * sref[1] ? 1 : 0;
    }
    T.info[0] = kC;
    T.info[1] = r;
    T.info[2] = ovf;
    if (ovf && T.overflow) atomicAdd(T.overflow, 1);
    if (T.rank) *T.rank = r;
  }
  // 4. Y_U^T = R_MJ^{-T} R_B[J,:]  and  Y_V = T1[:, J] R_MJ^{-1}; each thread
  //    solves for its own rows q (R_MJ[i][c] = row pivM[i] of the in-place
  //    factor at column pivM[c]), no barrier between the columns.  R_MJ is
  //    as ill-conditioned as the kept singular values are spread (up to
  //    1/tol): with double-double parts the solves run in double-double too,
  //    else the new factors lose their orthogonality (and C its accuracy)
  //    by about eps / tol.
  if (use_dd) {
    // The high parts of row q of Y_U and Y_V go to YU and YV, their low parts
    // to the slots of X (column q) and Z (row q) that this thread has read
    // already: no other thread reads those, and neither matrix is needed
    // after this step.  No per-thread arrays, hence no scratch memory (a
    // kernel with scratch cannot be dispatched once the device memory is
    // exhausted).
    for (int q = tid; q < K; q += HL_BLOCK) {
      double* yu = YU + q * RA_YS;
      double* yv = YV + q * RA_YS;
      for (int c = 0; c < r; ++c) {
        const int pc = pivM[c];
        dd u = {Xh[pivB[pc] * ks + q], Xl[pivB[pc] * ks + q]};
        dd v = {Zh[q * ks + pc], Zl[q * ks + pc]};
        for (int i = 0; i < c; ++i) {
          const int pi = pivM[i];
          const dd rmic = {Yh[pi * ks + pc], Yl[pi * ks + pc]};
          const dd sui = {yu[i], Xl[pivB[pi] * ks + q]};
          const dd svi = {yv[i], Zl[q * ks + pi]};
          u = dd_add(u, dd_neg(dd_mul(rmic, sui)));
          v = dd_add(v, dd_neg(dd_mul(rmic, svi)));
        }
        const dd dg = {Yh[pc * ks + pc], Yl[pc * ks + pc]};
        const dd su = dd_div(u, dg), sv = dd_div(v, dg);
        yu[c] = su.hi;
        yv[c] = sv.hi;
        Xl[pivB[pc] * ks + q] = su.lo;
        Zl[q * ks + pc] = sv.lo;
      }
      for (int c = r; c < RA_YS; ++c) {
        yu[c] = 0.0;
        yv[c] = 0.0;
      }
    }
    __syncthreads();
    return r;
  }
  for (int q = tid; q < K; q += HL_BLOCK) {
    double* yu = YU + q * RA_YS;
    double* yv = YV + q * RA_YS;
    for (int c = 0; c < r; ++c) {
      const int pc = pivM[c];
      const double dinv = 1.0 / Yh[pc * ks + pc];
      double u = Xh[pivB[pc] * ks + q];
      double v = Zh[q * ks + pc];
      for (int i = 0; i < c; ++i) {
        const double rmic = Yh[pivM[i] * ks + pc];
        u -= rmic * yu[i];
        v -= rmic * yv[i];
      }
      yu[c] = u * dinv;
      yv[c] = v * dinv;
    }
    for (int c = r; c < RA_YS; ++c) {
      yu[c] = 0.0;
      yv[c] = 0.0;
    }
  }
  __syncthreads();
  return r;
}

// LDS of the core for concatenations of at most ks columns: six (ks + 1)^2
// matrices (row stride ks + 1; the low parts of double-double only when the
// tolerance needs them, else three) and Y_U, Y_V
__host__ __device__ inline size_t radd_core_lds(int ks, bool dd_parts = true) {
  return ((dd_parts ? 6 : 3) * (size_t)(ks + 1) * (ks + 1) + 2 * (size_t)ks * RA_YS) * sizeof(double);
}
__host__ __device__ inline bool radd_needs_dd(double tol) { return radd_dd(tol); }

// Gram sums of the chunk partials (k_flush_gram) -> radd_core -> Y_U, Y_V to
// the target's workspace for k_flush_expand.  Dynamic LDS: radd_core_lds(ks).
__global__ void __launch_bounds__(HL_BLOCK) k_flush_core_fast(const LFlushTarget* tg, const Term* terms,
                                                              double tol, int ks) {
  extern __shared__ double smem[];
  const int ls = ks + 1;             // row stride of the LDS matrices
  const bool use_dd = radd_needs_dd(tol);
  // without double-double the low parts are neither read nor written; their
  // pointers alias the high parts
  double* Xh = smem;                 // G_B, then R_B (rows at pivot positions)
  double* Yh = Xh + ls * ls;         // G_A, then G_M / R_M
  double* Zh = Yh + ls * ls;         // T1 = G_A R_B^T (K x rB, row q col j at q * ls + j)
  double* Xl = use_dd ? Zh + ls * ls : Xh;
  double* Yl = use_dd ? Xl + ls * ls : Yh;
  double* Zl = use_dd ? Yl + ls * ls : Zh;
  double* YU = use_dd ? Zl + ls * ls : Zh + ls * ls;
  double* YV = YU + ks * RA_YS;
  __shared__ ColMap cm;
  __shared__ int pivB[KMAX], pivM[KMAX];
  __shared__ double sref[2];
  const LFlushTarget T = tg[blockIdx.x];
  const int tid = threadIdx.x;
  const int kC = T.rank ? *T.rank : 0;
  if (tid < 64) build_colmap(T, terms, kC, cm);
  __syncthreads();
  const int K = cm.K;
  const int Kc = T.Kcap;
  const int np = npairs(Kc);
  // Gram matrices (sum of the chunk partials), full symmetric storage
  for (int side = 0; side < 2; ++side) {
    double* Gh = side == 0 ? Yh : Xh;
    double* Gl = side == 0 ? Yl : Xl;
    const int nch = side == 0 ? T.nchA : T.nchB;
    const double* src = T.ws + (size_t)(side == 0 ? 0 : T.nchA) * np * 2;
    const int npk = npairs(K);
    for (int idx = tid; idx < npk; idx += HL_BLOCK) {
      int q = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
      while (q * (q + 1) / 2 > idx) --q;
      while ((q + 1) * (q + 2) / 2 <= idx) ++q;
      const int p = idx - q * (q + 1) / 2;
      dd s = {src[2 * idx], src[2 * idx + 1]};
      for (int c = 1; c < nch; c += 4) {
        double h[4], l[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          h[u] = 0.0;
          l[u] = 0.0;
          if (c + u < nch) {
            h[u] = src[(size_t)(c + u) * np * 2 + 2 * idx];
            l[u] = src[(size_t)(c + u) * np * 2 + 2 * idx + 1];
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) s = dd_add(s, {h[u], l[u]});
      }
      Gh[p * ls + q] = s.hi;
      Gh[q * ls + p] = s.hi;
      if (use_dd) {
        Gl[p * ls + q] = s.lo;
        Gl[q * ls + p] = s.lo;
      }
    }
  }
  __syncthreads();
  radd_core(T, kC, K, tol, ls, Xh, Xl, Yh, Yl, Zh, Zl, YU, YV, pivB, pivM, sref);
  // Y_U, Y_V (K x RA_YS each) to the workspace
  double* dst = T.ws + (size_t)(T.nchA + T.nchB) * np * 2;
  for (int e = tid; e < 2 * K * RA_YS; e += HL_BLOCK) dst[e] = e < K * RA_YS ? YU[e] : YV[e - K * RA_YS];
}


// U_new = A Y_U (side 0) or V_new = B Y_V (side 1) for rows [r0, r1)

// Column sources of the concatenated factors of a target (side 0: U side,
// side 1: V side): column j is sign * p[row - off] for row - off in [0, len),
// zero elsewhere.
struct RaddCols {
  const double* p[2][KMAX];
  int off[2][KMAX], len[2][KMAX];
  double sign[2][KMAX];
};

__device__ void radd_cols(const LFlushTarget& T, const Term* terms, const ColMap& cm, RaddCols& cs) {
  for (int e = threadIdx.x; e < 2 * cm.K; e += HL_BLOCK) {
    const int side = e / cm.K, j = e - side * cm.K;
    if (j < cm.kC) {
      cs.p[side][j] = side == 0 ? T.U + (size_t)T.m * j : T.V + (size_t)T.n * j;
      cs.off[side][j] = 0;
      cs.len[side][j] = side == 0 ? T.m : T.n;
      cs.sign[side][j] = 1.0;
    } else {
      int t = 0;
      while (j >= cm.off[t + 1]) ++t;
      const Term& tm = terms[T.tbeg + cm.tb + t];
      const int c = j - cm.off[t];
      cs.p[side][j] = side == 0 ? tm.U + (size_t)tm.ldu * c : tm.W + (size_t)tm.ldw * c;
      cs.off[side][j] = side == 0 ? tm.ro : tm.co;
      cs.len[side][j] = side == 0 ? tm.mr : tm.nc;
      cs.sign[side][j] = side == 0 ? tm.sign : 1.0;
    }
  }
}

// rows [base, base + 64) of one side, all K columns: radd_fetch_tile issues
// the loads into registers (zero past the rows), radd_store_tile writes them
// to tile[rr + RA_TS j]; fetching the next block before working on the current
// one keeps a block's loads in flight during the work
constexpr int RA_NE = 64 * KMAX / HL_BLOCK;
__device__ __forceinline__ void radd_fetch_tile(const RaddCols& cs, int side, int base, int rows, int K,
                                                double (&v)[RA_NE]) {
#pragma unroll
  for (int u = 0; u < RA_NE; ++u) {
    const int e = threadIdx.x + u * HL_BLOCK;
    const int rr = e & 63, j = e >> 6;   // j is uniform across a wavefront
    v[u] = 0.0;
    // only columns j < K have sources (radd_cols writes no others, so with
    // K = 0 nothing is loaded); a column of zero length loads nothing
    if (j < K) {
      const int len = cs.len[side][j];
      if (len > 0) {
        int i = base + rr - cs.off[side][j];
        const bool ok = rr < rows && i >= 0 && i < len;
        i = min(max(i, 0), len - 1);   // in bounds for every lane: loads stay unconditional
        const double x = cs.p[side][j][i];
        v[u] = ok ? cs.sign[side][j] * x : 0.0;
      }
    }
  }
}
constexpr int RA_TS = 65;   // column stride of a staged row block (odd: no LDS bank conflicts across columns)
__device__ __forceinline__ void radd_store_tile(const double (&v)[RA_NE], int K, double* tile) {
#pragma unroll
  for (int u = 0; u < RA_NE; ++u) {
    const int e = threadIdx.x + u * HL_BLOCK;
    if ((e >> 6) < K) tile[(e & 63) + RA_TS * (e >> 6)] = v[u];
  }
}

// Gram of staged 64-row blocks on the matrix cores: the upper 16 x 16 tiles
// (TI <= TJ) of the K x K Gram, at most 3 per wavefront of a 256-thread
// block; per block 16 steps of v_mfma_f64_16x16x4f64 with A = tile^T
// (A[i][k] in lane i + 16 k) and B = tile (B[k][j] in lane j + 16 k); D[i][j]
// sits in lane 16 (i % 4) + j, register i / 4.  Columns >= K count as zero.
struct GramTiles {
  int tI[3], tJ[3], nup;
  double4v acc[3];
};
__device__ __forceinline__ void gram_tiles_init(GramTiles& g, int K, int wv) {
  const int nT = (K + 15) / 16;
  g.nup = nT * (nT + 1) / 2;
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    g.acc[u] = double4v{0.0, 0.0, 0.0, 0.0};
    int idx = wv + 4 * u, a = 0;
    while (a < nT && idx >= nT - a) {   // upper tile number idx -> (a, b)
      idx -= nT - a;
      ++a;
    }
    g.tI[u] = a;
    g.tJ[u] = a + idx;
  }
}
__device__ __forceinline__ void gram_tiles_add(GramTiles& g, const double* tile, int K, int wv, int lane) {
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    if (wv + 4 * u >= g.nup) break;
    const int ca = 16 * g.tI[u] + (lane & 15), cb = 16 * g.tJ[u] + (lane & 15);
    const double* ta = tile + RA_TS * min(ca, K - 1);
    const double* tb = tile + RA_TS * min(cb, K - 1);
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const int rr = 4 * kk + (lane >> 4);
      const double a = ca < K ? ta[rr] : 0.0;
      const double b = cb < K ? tb[rr] : 0.0;
      g.acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, g.acc[u], 0, 0, 0);
    }
  }
}
// store(p, q, value) once per pair p <= q < K
template <class F>
__device__ __forceinline__ void gram_tiles_store(const GramTiles& g, int K, int wv, int lane, F&& store) {
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    if (wv + 4 * u >= g.nup) break;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = 16 * g.tI[u] + 4 * r + (lane >> 4), q = 16 * g.tJ[u] + (lane & 15);
      if (p < K && q < K && (g.tI[u] < g.tJ[u] || p <= q)) store(p, q, g.acc[u][r]);
    }
  }
}

// rows of a staged 64-row block times Y (K x r, row stride RA_YS) on the
// matrix cores: wavefront wv takes rows 16 wv .. 16 wv + 15 and the (at
// most two) 16-column tiles of the r columns; out[row + ld c] for the
// block's first `rows` rows
__device__ __forceinline__ void expand_block_mfma(const double* tile, const double* Y, int K, int r, int rows,
                                                  int wv, int lane, double* out, size_t ld) {
  const int nC = (r + 15) / 16;
  double4v eacc[2] = {double4v{0.0, 0.0, 0.0, 0.0}, double4v{0.0, 0.0, 0.0, 0.0}};
  const double* ta = tile + 16 * wv + (lane & 15);
  for (int kk = 0; kk < (K + 3) / 4; ++kk) {
    const int j = 4 * kk + (lane >> 4);
    const double a = j < K ? ta[RA_TS * j] : 0.0;
#pragma unroll
    for (int cj = 0; cj < 2; ++cj) {
      if (cj >= nC) break;
      const double b = j < K ? Y[j * RA_YS + 16 * cj + (lane & 15)] : 0.0;
      eacc[cj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, eacc[cj], 0, 0, 0);
    }
  }
#pragma unroll
  for (int cj = 0; cj < 2; ++cj) {
    if (cj >= nC) break;
    const int c = 16 * cj + (lane & 15);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int row = 16 * wv + 4 * q + (lane >> 4);
      if (row < rows && c < r) out[row + ld * c] = eacc[cj][q];
    }
  }
}

// Partial Gram of rows [r0, r1) of one side of a bucketed rounded
// addition, packed upper triangle (double-double below RADD_DD_TOL, else on the
// matrix cores).
__global__ void __launch_bounds__(HL_BLOCK) k_flush_gram(const LFlushTarget* tg, const Term* terms,
                                                         const ChunkItem* items, double tol) {
  __shared__ ColMap cm;
  __shared__ RaddCols cs;
  __shared__ double tile[RA_TS * KMAX];   // 64 x K, column stride RA_TS
  const ChunkItem it = items[blockIdx.x];
  const LFlushTarget T = tg[it.tgt];
  if (threadIdx.x < 64) build_colmap(T, terms, T.rank ? *T.rank : 0, cm);
  __syncthreads();
  radd_cols(T, terms, cm, cs);
  __syncthreads();
  const int K = cm.K;
  const int Kc = T.Kcap;
  double* dst = T.ws + (size_t)(it.side == 0 ? it.chunk : T.nchA + it.chunk) * npairs(Kc) * 2;
  double v[RA_NE];
  radd_fetch_tile(cs, it.side, it.r0, min(64, it.r1 - it.r0), K, v);
  if (!radd_needs_dd(tol)) {
    // on the matrix cores (low parts zero)
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
    GramTiles gt;
    gram_tiles_init(gt, K, wv);
    for (int base = it.r0; base < it.r1; base += 64) {
      __syncthreads();
      radd_store_tile(v, K, tile);
      __syncthreads();
      if (base + 64 < it.r1) radd_fetch_tile(cs, it.side, base + 64, min(64, it.r1 - base - 64), K, v);
      gram_tiles_add(gt, tile, K, wv, lane);
    }
    gram_tiles_store(gt, K, wv, lane, [&](int pp, int qq, double x) {
      const int idx = pair_index(pp, qq);
      dst[2 * idx] = x;
      dst[2 * idx + 1] = 0.0;
    });
    return;
  }
  const int np = npairs(K);
  constexpr int PPT = (KMAX * (KMAX + 1) / 2 + HL_BLOCK - 1) / HL_BLOCK;  // pairs per thread
  dd accv[PPT];
  int pp[PPT], qq[PPT];
  for (int u = 0; u < PPT; ++u) {
    accv[u] = {0.0, 0.0};
    int idx = threadIdx.x + u * HL_BLOCK;
    pp[u] = qq[u] = -1;
    if (idx < np) {
      int q = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
      while (q * (q + 1) / 2 > idx) --q;
      while ((q + 1) * (q + 2) / 2 <= idx) ++q;
      pp[u] = idx - q * (q + 1) / 2;
      qq[u] = q;
    }
  }
  for (int base = it.r0; base < it.r1; base += 64) {
    __syncthreads();
    radd_store_tile(v, K, tile);
    __syncthreads();
    if (base + 64 < it.r1) radd_fetch_tile(cs, it.side, base + 64, min(64, it.r1 - base - 64), K, v);
    for (int u = 0; u < PPT; ++u) {
      if (pp[u] < 0) continue;
      const double* a = tile + RA_TS * pp[u];
      const double* b = tile + RA_TS * qq[u];
      dd s = accv[u];
      for (int rr = 0; rr < 64; ++rr) s = dd_add(s, dd_mul_d(a[rr], b[rr]));
      accv[u] = s;
    }
  }
  for (int u = 0; u < PPT; ++u) {
    if (pp[u] < 0) continue;
    int idx = pair_index(pp[u], qq[u]);
    dst[2 * idx] = accv[u].hi;
    dst[2 * idx + 1] = accv[u].lo;
  }
}

// New factor rows [r0, r1) of one side of a bucketed rounded addition.
__global__ void __launch_bounds__(HL_BLOCK) k_flush_expand(const LFlushTarget* tg, const Term* terms,
                                                           const ChunkItem* items) {
  __shared__ ColMap cm;
  __shared__ RaddCols cs;
  __shared__ double Y[KMAX * RA_YS];
  __shared__ double tile[RA_TS * KMAX];
  const ChunkItem it = items[blockIdx.x];
  const LFlushTarget T = tg[it.tgt];
  const int kC = T.info[0], r = T.info[1];
  if (threadIdx.x < 64) build_colmap(T, terms, kC, cm);
  __syncthreads();
  radd_cols(T, terms, cm, cs);
  const int K = cm.K, Kc = T.Kcap;
  const int np = npairs(Kc);
  const double* Ys = T.ws + (size_t)(T.nchA + T.nchB) * np * 2 + (it.side == 0 ? 0 : (size_t)K * RA_YS);
  for (int e = threadIdx.x; e < K * RA_YS; e += HL_BLOCK) Y[e] = Ys[e];
  __syncthreads();
  // new factor rows [r0, r1) = concatenation rows times Y (row-local: the
  // next block is fetched before this one is written)
  double* out = it.side == 0 ? T.U : T.V;
  const size_t ld = it.side == 0 ? T.m : T.n;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  double v[RA_NE];
  radd_fetch_tile(cs, it.side, it.r0, min(64, it.r1 - it.r0), K, v);
  for (int base = it.r0; base < it.r1; base += 64) {
    const int rows = min(64, it.r1 - base);
    __syncthreads();
    radd_store_tile(v, K, tile);
    __syncthreads();
    if (base + 64 < it.r1) radd_fetch_tile(cs, it.side, base + 64, min(64, it.r1 - base - 64), K, v);
    expand_block_mfma(tile, Y, K, r, rows, wv, lane, out + base, ld);
  }
}

// Whole rounded additions in one workgroup for a target of at most
// GRAM_CHUNK rows on each side and any number of terms: the terms are taken
// in concatenations of at most ks columns (actual ranks, known only here),
// each one a rounded addition into the target: Gram matrices straight from
// the factors, radd_core, then the new factors in place, 64 rows at a time
// (a row block is staged in LDS before any of its rows is overwritten).
// smem: radd_fused_lds(ks) bytes of dynamic LDS.
__device__ __forceinline__ void radd_fused_target(const LFlushTarget& T, const Term* terms, double tol, int ks,
                                                  double* smem) {
  const int ls = ks + 1;   // row stride of the LDS matrices
  const bool use_dd = radd_needs_dd(tol);
  // with double-double parts: X, Y, Z high and low (the 64 x K tile of a
  // row block lives in Z, 2 ls^2 >= RA_TS ks doubles for ks >= 32); without:
  // X, Y high only (low pointers alias them, never written) and Z sized for
  // the tile
  double *Xh, *Xl, *Yh, *Yl, *Zh, *Zl, *YU;
  if (use_dd) {
    Xh = smem;
    Xl = Xh + ls * ls;
    Yh = Xl + ls * ls;
    Yl = Yh + ls * ls;
    Zh = Yl + ls * ls;
    Zl = Zh + ls * ls;
    YU = Zl + ls * ls;
  } else {
    Xh = smem;
    Xl = Xh;
    Yh = Xh + ls * ls;
    Yl = Yh;
    Zh = Yh + ls * ls;
    Zl = Zh;
    YU = Zh + max(ls * ls, RA_TS * ks);
  }
  double* YV = YU + ks * RA_YS;
  double* tile = Zh;   // 64 x K, column stride RA_TS
  __shared__ ColMap cm;
  __shared__ RaddCols cs;
  __shared__ int pivB[KMAX], pivM[KMAX];
  __shared__ double sref[2];
  const int tid = threadIdx.x;
  constexpr int PPT = (KMAX * (KMAX + 1) / 2 + HL_BLOCK - 1) / HL_BLOCK;
  int r = T.rank ? *T.rank : 0;
  // the term list in concatenations of at most ks columns, each one a whole
  // rounded addition into the target
  for (int t0 = 0; t0 < T.tcount;) {
    __syncthreads();
    if (tid < 64) build_colmap_chunk(T, terms, r, t0, ks, cm);
    __syncthreads();
    const int K = cm.K, kC = r;
    if (K > ks) {
      // a single term wider than the LDS matrices (excluded by the planner):
      // flag it and leave the target
      if (tid == 0) {
        T.info[2] = 1;
        if (T.overflow) atomicAdd(T.overflow, 1);
      }
      break;
    }
    radd_cols(T, terms, cm, cs);
    __syncthreads();   // the column sources are read by every thread below
    const int np = npairs(K);
    int pp[PPT], qq[PPT];
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int idx = tid + u * HL_BLOCK;
      pp[u] = qq[u] = 0;
      if (idx < np) {
        int q = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
        while (q * (q + 1) / 2 > idx) --q;
        while ((q + 1) * (q + 2) / 2 <= idx) ++q;
        pp[u] = idx - q * (q + 1) / 2;
        qq[u] = q;
      }
    }
    // an empty target whose terms are unit-column pieces: G_B = I is known
    const bool b_orth = T.borth && kC == 0;
    const int nside = b_orth ? 1 : 2;
    double v[RA_NE];
    radd_fetch_tile(cs, 0, 0, min(64, T.m), K, v);
    for (int side = 0; side < nside; ++side) {
      const int len = side == 0 ? T.m : T.n;
      double* Gh = side == 0 ? Yh : Xh;
      double* Gl = side == 0 ? Yl : Xl;
      if (!use_dd) {
        // Gram on the matrix cores
        const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
        GramTiles gt;
        gram_tiles_init(gt, K, wv);
        for (int base = 0; base < len; base += 64) {
          __syncthreads();
          radd_store_tile(v, K, tile);
          __syncthreads();
          if (base + 64 < len)
            radd_fetch_tile(cs, side, base + 64, min(64, len - base - 64), K, v);
          else if (side + 1 < nside)
            radd_fetch_tile(cs, 1, 0, min(64, T.n), K, v);
          gram_tiles_add(gt, tile, K, wv, lane);
        }
        gram_tiles_store(gt, K, wv, lane, [&](int p, int q, double x) {
          Gh[p * ls + q] = x;
          Gh[q * ls + p] = x;
        });
        continue;
      }
      dd accv[PPT];
#pragma unroll
      for (int u = 0; u < PPT; ++u) accv[u] = {0.0, 0.0};
      for (int base = 0; base < len; base += 64) {
        __syncthreads();
        radd_store_tile(v, K, tile);
        __syncthreads();
        // next block: this side's, else the first of the V side
        if (base + 64 < len)
          radd_fetch_tile(cs, side, base + 64, min(64, len - base - 64), K, v);
        else if (side + 1 < nside)
          radd_fetch_tile(cs, 1, 0, min(64, T.n), K, v);
#pragma unroll
        for (int u = 0; u < PPT; ++u) {
          if (tid + u * HL_BLOCK >= np) continue;
          const double* a = tile + RA_TS * pp[u];
          const double* b = tile + RA_TS * qq[u];
          dd acc = accv[u];
          for (int rr = 0; rr < 64; ++rr) acc = dd_add(acc, dd_mul_d(a[rr], b[rr]));
          accv[u] = acc;
        }
      }
#pragma unroll
      for (int u = 0; u < PPT; ++u) {
        if (tid + u * HL_BLOCK >= np) continue;
        Gh[pp[u] * ls + qq[u]] = accv[u].hi;
        Gh[qq[u] * ls + pp[u]] = accv[u].hi;
        Gl[pp[u] * ls + qq[u]] = accv[u].lo;
        Gl[qq[u] * ls + pp[u]] = accv[u].lo;
      }
    }
    __syncthreads();
    r = radd_core(T, kC, K, tol, ls, Xh, Xl, Yh, Yl, Zh, Zl, YU, YV, pivB, pivM, sref, b_orth);
    // new factors: U_new = A Y_U, V_new = B Y_V
    radd_fetch_tile(cs, 0, 0, min(64, T.m), K, v);
    for (int side = 0; side < 2; ++side) {
      const int len = side == 0 ? T.m : T.n;
      double* out = side == 0 ? T.U : T.V;
      const double* Y = side == 0 ? YU : YV;
      for (int base = 0; base < len; base += 64) {
        const int rows = min(64, len - base);
        __syncthreads();
        radd_store_tile(v, K, tile);
        __syncthreads();
        // the next block is read before this one is overwritten: rows differ
        if (base + 64 < len)
          radd_fetch_tile(cs, side, base + 64, min(64, len - base - 64), K, v);
        else if (side == 0)
          radd_fetch_tile(cs, 1, 0, min(64, T.n), K, v);
        expand_block_mfma(tile, Y, K, r, rows, __builtin_amdgcn_readfirstlane(tid >> 6), tid & 63, out + base,
                          (size_t)len);
      }
    }
    t0 += cm.nt;
  }
}

__host__ __device__ inline size_t radd_fused_lds(int ks, bool dd_parts = true) {
  // with double-double parts the Gram tile (64 x ks) lives in Z (2 ks^2
  // doubles): ks >= 32; without, Z is sized for the tile
  const int k = ks < 32 ? 32 : ks;
  if (dd_parts) return radd_core_lds(k);
  const size_t ls2 = (size_t)(k + 1) * (k + 1);
  return (2 * ls2 + std::max(ls2, (size_t)RA_TS * k) + 2 * (size_t)k * RA_YS) * sizeof(double);
}

// ---------------------------------------------------------------------------
// dense targets, products, copies, leaf factorisation
// ---------------------------------------------------------------------------
// Dense target (at most 64 x 64): D += sum of its terms, accumulated in
// the matrix-core registers of four 32 x 32 quadrants (one per wavefront).
// Product and low-rank terms are taken in 32-column slices of the inner
// dimension staged in LDS at target positions (zero outside the term's rows
// / columns), the next slice fetched into registers while the current one
// is used.
constexpr int DF_KC = 32;
constexpr int DF_NE = 2 * 64 * DF_KC / HL_BLOCK;   // staged values per thread and slice

__device__ __forceinline__ int term_inner(const Term& tm) {
  return tm.dense == 2 ? tm.kfix : term_rank(tm);
}

// slice [q0, q0 + DF_KC) of the inner dimension: element e < 64 * DF_KC is
// A(i, q) (i = e % 64), the rest B(q, j) (j = e' % 64), zero outside the term
__device__ __forceinline__ void df_fetch(const Term& tm, int kin, int q0, double (&v)[DF_NE]) {
  // unconditional loads at clamped (in-bounds) indices, so that all of a
  // thread's loads are in flight together; masked values become zero
#pragma unroll
  for (int u = 0; u < DF_NE; ++u) {
    const int e = threadIdx.x + u * HL_BLOCK;
    const bool left = e < 64 * DF_KC;
    const int f = left ? e : e - 64 * DF_KC;
    const int x = f & 63, q = q0 + (f >> 6);
    // a term of inner dimension 0 (rank 0) or of no rows / columns loads
    // nothing: the clamped indices below need at least one element
    const bool live = kin > 0 && tm.mr > 0 && tm.nc > 0;
    const int qc = min(q, kin - 1);
    double val = 0.0;
    bool ok = false;
    if (live) {
      if (left) {
        const int i = x - tm.ro;
        ok = i >= 0 && i < tm.mr && q < kin;
        val = tm.U[min(max(i, 0), tm.mr - 1) + (size_t)tm.ldu * qc];
        val *= tm.sign;
      } else {
        const int j = x - tm.co;
        ok = j >= 0 && j < tm.nc && q < kin;
        const int jc = min(max(j, 0), tm.nc - 1);
        val = tm.dense == 2 ? tm.W[qc + (size_t)tm.ldw * jc] : tm.W[jc + (size_t)tm.ldw * qc];
      }
    }
    v[u] = ok ? val : 0.0;
  }
}

// 64 x 64 block products on the matrix cores: wavefront wv of a 256-thread
// block owns the 32 x 32 quadrant of row tiles 2 (wv >> 1) + {0, 1} and
// column tiles 2 (wv & 1) + {0, 1}; acc[a][b][v] is C[i][j] with
// i = 16 (2 (wv >> 1) + a) + 4 v + lane / 16, j = 16 (2 (wv & 1) + b) + lane % 16.
// One step of v_mfma_f64_16x16x4f64 per tile and 4 inner indices, with
// A(i, q) at As[i + 64 q] in lane i % 16 + 16 (q % 4) and B(q, j) at
// Bs[j + 64 q] in lane j % 16 + 16 (q % 4).
struct Quad64 {
  double4v acc[2][2];
};
__device__ __forceinline__ int quad_row(int wv, int a, int v, int lane) {
  return 16 * (2 * (wv >> 1) + a) + 4 * v + (lane >> 4);
}
__device__ __forceinline__ int quad_col(int wv, int b, int lane) { return 16 * (2 * (wv & 1) + b) + (lane & 15); }
// C += A(:, 0 .. 4 n4) B(0 .. 4 n4, :) from the staged operands
__device__ __forceinline__ void quad_mma(Quad64& Q, const double* As, const double* Bs, int n4, int wv,
                                         int lane) {
  const double* pa = As + 32 * (wv >> 1) + (lane & 15) + 64 * (lane >> 4);
  const double* pb = Bs + 32 * (wv & 1) + (lane & 15) + 64 * (lane >> 4);
  for (int kk = 0; kk < n4; ++kk) {
    const double a0 = pa[256 * kk], a1 = pa[256 * kk + 16];
    const double b0 = pb[256 * kk], b1 = pb[256 * kk + 16];
    Q.acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, Q.acc[0][0], 0, 0, 0);
    Q.acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, Q.acc[0][1], 0, 0, 0);
    Q.acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, Q.acc[1][0], 0, 0, 0);
    Q.acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, Q.acc[1][1], 0, 0, 0);
  }
}

// As, Bs: DF_KC * 64 doubles each of LDS, A(i, q) at i + 64 q, B(q, j) at j + 64 q
__device__ __forceinline__ void flush_dense_item(const DFlushItem& it, const Term* terms, double* As, double* Bs) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  Quad64 Q;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = quad_row(wv, a, v, lane), j = quad_col(wv, b, lane);
        Q.acc[a][b][v] = (i < it.m && j < it.n) ? it.D[i + (size_t)it.ldd * j] : 0.0;
      }
  for (int t = 0; t < it.tcount; ++t) {
    const Term tm = terms[it.tbeg + t];
    if (tm.dense == 1) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int i = quad_row(wv, a, v, lane) - tm.ro, j = quad_col(wv, b, lane) - tm.co;
            if (i >= 0 && i < tm.mr && j >= 0 && j < tm.nc) Q.acc[a][b][v] += tm.sign * tm.U[i + (size_t)tm.ldu * j];
          }
      continue;
    }
    const int kin = term_inner(tm);
    double v[DF_NE];
    if (kin > 0) df_fetch(tm, kin, 0, v);
    for (int q0 = 0; q0 < kin; q0 += DF_KC) {
      __syncthreads();
#pragma unroll
      for (int u = 0; u < DF_NE; ++u) {
        const int e = tid + u * HL_BLOCK;
        if (e < 64 * DF_KC) As[e] = v[u];
        else Bs[e - 64 * DF_KC] = v[u];
      }
      __syncthreads();
      if (q0 + DF_KC < kin) df_fetch(tm, kin, q0 + DF_KC, v);
      // inner indices past kin were staged as zeros
      quad_mma(Q, As, Bs, (min(DF_KC, kin - q0) + 3) / 4, wv, lane);
    }
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = quad_row(wv, a, v, lane), j = quad_col(wv, b, lane);
        if (i < it.m && j < it.n) it.D[i + (size_t)it.ldd * j] = Q.acc[a][b][v];
      }
}

__global__ void __launch_bounds__(HL_BLOCK) k_flush_dense(const DFlushItem* items, const Term* terms) {
  __shared__ double As[DF_KC * 64], Bs[DF_KC * 64];
  flush_dense_item(items[blockIdx.x], terms, As, Bs);
}

// The fused rounded additions of a batch (blocks 0 .. ntg-1) and, in the
// same launch, the batch's dense-target flushes (blocks ntg ..): the two
// write disjoint leaves and read none of each other's, so they overlap
// instead of running back to back.  Dynamic LDS: radd_fused_dyn_lds(ks, tol).
__global__ void __launch_bounds__(HL_BLOCK) k_radd_fused(const LFlushTarget* tg, int ntg, const Term* terms,
                                                         double tol, int ks, const DFlushItem* dfl,
                                                         const Term* dterms) {
  extern __shared__ double smem[];
  if ((int)blockIdx.x >= ntg) {
    flush_dense_item(dfl[blockIdx.x - ntg], dterms, smem, smem + DF_KC * 64);
    return;
  }
  radd_fused_target(tg[blockIdx.x], terms, tol, ks, smem);
}

// P = A B for blocks of at most 64 x 64 (inner dimension at most 64), on
// the matrix cores; the operands are staged zero-padded to 64 x 64
__global__ void __launch_bounds__(HL_BLOCK) k_dense_prod(const DProdItem* items) {
  __shared__ double As[64 * 64], Bs[64 * 64];   // A(i, q) at i + 64 q, B(q, j) at j + 64 q
  const DProdItem it = items[blockIdx.x];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int e = tid; e < 64 * 64; e += HL_BLOCK) {
    const int i = e & 63, q = e >> 6;
    As[e] = (i < it.m && q < it.k) ? it.A[i + (size_t)it.lda * q] : 0.0;
  }
  for (int e = tid; e < 64 * 64; e += HL_BLOCK) {
    const int q = e & 63, j = e >> 6;   // coalesced along q in global memory
    Bs[j + 64 * q] = (q < it.k && j < it.n) ? it.B[q + (size_t)it.ldb * j] : 0.0;
  }
  __syncthreads();
  Quad64 Q;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) Q.acc[a][b] = double4v{0.0, 0.0, 0.0, 0.0};
  quad_mma(Q, As, Bs, (it.k + 3) / 4, wv, lane);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = quad_row(wv, a, v, lane), j = quad_col(wv, b, lane);
        if (i < it.m && j < it.n) it.P[i + (size_t)it.ldp * j] = Q.acc[a][b][v];
      }
}

__global__ void __launch_bounds__(HL_BLOCK) k_copy_leaf(const CopyItem* items) {
  const CopyItem it = items[blockIdx.x];
  if (it.dense && it.expand) {
    const int k = (it.A && it.rank) ? *it.rank : 0;
    const int tot = it.m * it.n;
    for (int e = threadIdx.x; e < tot; e += HL_BLOCK) {
      const int i = e % it.m, j = e / it.m;
      double v = 0.0;
      for (int p = 0; p < k; ++p) v += it.A[i + (size_t)it.m * p] * it.B[j + (size_t)it.n * p];
      it.dA[e] = it.scale * v;
    }
    return;
  }
  if (it.dense) {
    const int tot = it.m * it.n;
    for (int e = threadIdx.x; e < tot; e += HL_BLOCK) {
      double v = it.A ? it.scale * it.A[e] : 0.0;
      if (it.add_identity && (e % it.m) == (e / it.m)) v += 1.0;
      it.dA[e] = v;
      if (it.zA) it.zA[e] = 0.0;   // move: each element is read before it is cleared, by the same thread
    }
    return;
  }
  const int k = (it.A && it.rank) ? *it.rank : 0;
  for (int e = threadIdx.x; e < it.m * k; e += HL_BLOCK) it.dA[e] = it.scale * it.A[e];
  for (int e = threadIdx.x; e < it.n * k; e += HL_BLOCK) it.dB[e] = it.B[e];
  if (threadIdx.x == 0 && it.drank) *it.drank = k;
  if (it.zrank) {
    __syncthreads();   // every thread has read the source rank
    if (threadIdx.x == 0) *it.zrank = 0;
  }
}

// LU without pivoting of a diagonal leaf (in place), then the inverses of the
// unit-lower factor and of the upper factor.
__global__ void __launch_bounds__(HL_BLOCK) k_getrf_inv(const GetrfItem* items, int32_t* zero_pivot) {
  // column stride 65 for both arrays: no LDS bank conflicts when threads
  // walk different columns
  __shared__ double Ap[64 * 65];
  __shared__ double X[64 * 65];
  const GetrfItem it = items[blockIdx.x];
  const int m = it.m;
#define A(i, j) Ap[(i) + 65 * (j)]
  for (int e = threadIdx.x; e < m * m; e += HL_BLOCK) A(e % m, e / m) = it.LU[e];
  __syncthreads();
  for (int kk = 0; kk < m; ++kk) {
    const double piv = A(kk, kk);
    if (piv == 0.0) {
      if (threadIdx.x == 0) atomicAdd(zero_pivot, 1);
      return;
    }
    for (int i = kk + 1 + threadIdx.x; i < m; i += HL_BLOCK) A(i, kk) /= piv;
    __syncthreads();
    const int rem = m - kk - 1;
    for (int e = threadIdx.x; e < rem * rem; e += HL_BLOCK) {
      int i = kk + 1 + e % rem, j = kk + 1 + e / rem;
      A(i, j) -= A(i, kk) * A(kk, j);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < m * m; e += HL_BLOCK) it.LU[e] = A(e % m, e / m);
  // inverse of the unit lower factor, right-looking: X = I; for each k,
  // X[i, :] -= L[i, k] X[k, :] for i > k (all (i, c) in parallel)
  for (int e = threadIdx.x; e < m * m; e += HL_BLOCK) X[(e % m) + 65 * (e / m)] = (e % m) == (e / m) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = 0; k < m - 1; ++k) {
    const int rem = m - k - 1;
    for (int e = threadIdx.x; e < rem * (k + 1); e += HL_BLOCK) {
      const int i = k + 1 + e % rem, c = e / rem;   // X[k, c] = 0 for c > k
      X[i + 65 * c] -= A(i, k) * X[k + 65 * c];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < m * m; e += HL_BLOCK) it.Li[e] = X[(e % m) + 65 * (e / m)];
  __syncthreads();
  // inverse of the upper factor, right-looking from the bottom: X = I; for
  // k = m-1 .. 0: X[k, :] /= U[k, k]; X[i, :] -= U[i, k] X[k, :] for i < k
  for (int e = threadIdx.x; e < m * m; e += HL_BLOCK) X[(e % m) + 65 * (e / m)] = (e % m) == (e / m) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = m - 1; k >= 0; --k) {
    const double inv = 1.0 / A(k, k);
    for (int c = threadIdx.x; c < m; c += HL_BLOCK) X[k + 65 * c] *= inv;
    __syncthreads();
    for (int e = threadIdx.x; e < k * m; e += HL_BLOCK) {
      const int i = e % k, c = e / k;
      X[i + 65 * c] -= A(i, k) * X[k + 65 * c];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < m * m; e += HL_BLOCK) it.Ui[e] = X[(e % m) + 65 * (e / m)];
#undef A
}

// ---------------------------------------------------------------------------
// Dense diagonal block of up to 2 x 2 leaf tiles (App. B.3 at the bottom of
// the recursion): LU without pivoting, then the inverses of the unit lower
// factor L and of the upper factor U, all in one workgroup of 1024 threads.
// The block, padded with the identity to LUINV_N = 128, lives in registers
// with a cyclic layout: thread (ty, tx) owns rows ty + 32 r and columns
// tx + 32 c (r, c < 4), so the owner of column k holds it in register
// column k / 32 -- a constant over 32 consecutive steps, which keeps every
// register index static.  One pass of n elimination steps advances the LU
// and both inverses together, each step publishing two columns and two rows
// through LDS (double buffered, one barrier per step): X = L^{-1} by the
// step's row operations applied to I, Y = U'^{-1} (U' = D^{-1} U, unit
// upper) by its column operations applied to I, U^{-1} = Y D^{-1}; X is
// strictly lower and Y strictly upper, so both share one register array.
// ---------------------------------------------------------------------------
constexpr int LI_G = 32;                  // thread grid is LI_G x LI_G
constexpr int LI_T = LI_G * LI_G;         // 1024 threads
constexpr int LI_R = LUINV_N / LI_G;      // 4 x 4 entries per thread
constexpr int LI_S = LUINV_N + 1;         // LDS stage stride (odd: fewer bank conflicts)

size_t luinv_lds_bytes() { return sizeof(double) * ((size_t)LUINV_N * LI_S + 9 * LUINV_N); }

__global__ void __launch_bounds__(LI_T) k_lu_inv(const LuInvItem* items, int32_t* zero_pivot) {
  extern __shared__ double lds[];
  double* stage = lds;                          // LUINV_N x LI_S
  double* pub = lds + (size_t)LUINV_N * LI_S;   // [2][4][LUINV_N]
  double* dinv = pub + 8 * LUINV_N;             // 1 / U[k, k]
  const LuInvItem it = items[blockIdx.x];
  const int m1 = it.m1, m2 = it.m2, n = m1 + m2;
  const int tid = threadIdx.x, ty = tid / LI_G, tx = tid % LI_G;

  // every thread's 16 loads are issued before the first LDS store: a fixed
  // trip count and no branches (the source block and offset are selected;
  // an entry of the identity padding loads A11[0], which always exists, and
  // discards it), so nothing waits between the loads
  {
    constexpr int LI_E = LUINV_N * LUINV_N / LI_T;
    double vals[LI_E];
#pragma unroll
    for (int u = 0; u < LI_E; ++u) {
      const int e = tid + u * LI_T;
      const int i = e % LUINV_N, j = e / LUINV_N;
      const bool in = i < n && j < n, top = i < m1, left = j < m1;
      const double* src = !in ? it.A11 : (top ? (left ? it.A11 : it.A12) : (left ? it.A21 : it.A22));
      const size_t off =
          !in ? 0 : (size_t)(top ? i : i - m1) + (size_t)(top ? m1 : m2) * (size_t)(left ? j : j - m1);
      const double x = src[off];
      vals[u] = in ? x : (i == j ? 1.0 : 0.0);
    }
#pragma unroll
    for (int u = 0; u < LI_E; ++u) {
      const int e = tid + u * LI_T;
      stage[(e % LUINV_N) + LI_S * (e / LUINV_N)] = vals[u];
    }
  }
  __syncthreads();
  double a[LI_R][LI_R], z[LI_R][LI_R];
#pragma unroll
  for (int r = 0; r < LI_R; ++r)
#pragma unroll
    for (int c = 0; c < LI_R; ++c) {
      a[r][c] = stage[(ty + LI_G * r) + LI_S * (tx + LI_G * c)];
      z[r][c] = 0.0;
    }

  // One pass of n elimination steps.  Step k publishes column k of the
  // active matrix (rows >= k), its row k (columns > k), row k of X = L^{-1}
  // (columns < k) and column k of Y = U'^{-1} (rows < k), all final at step
  // k, then every thread applies
  //   A[i, j] -= l_ik u_kj           (i, j > k; the Schur complement)
  //   X[i, c] -= l_ik X[k, c]         (i > k, c <= k; row operations on I)
  //   Y[r, j] -= Y[r, k] u_kj / u_kk  (r <= k, j > k; column operations on I)
  // with l_ik = A[i, k] / u_kk, X[k, k] = Y[k, k] = 1.  X (strictly lower)
  // and Y (strictly upper) share the register array z.
  bool zp = false;
#pragma unroll
  for (int cb = 0; cb < LI_R; ++cb) {
    const int kend = min(n, LI_G * (cb + 1));
    for (int k = LI_G * cb; k < kend; ++k) {
      const int kk = k - LI_G * cb;
      double* col = pub + (k & 1) * 4 * LUINV_N;
      double* row = col + LUINV_N;
      double* xr = row + LUINV_N;
      double* yc = xr + LUINV_N;
      // Row i = ty + 32 r of register block r lies below k for r > cb and
      // above it for r < cb (likewise columns), so only block cb compares
      // at run time; the pivot's owner forms 1 / U[k, k] once for all.
      if (tx == kk) {
#pragma unroll
        for (int r = 0; r < LI_R; ++r) {
          const int i = ty + LI_G * r;
          if (r > cb || (r == cb && ty >= kk)) col[i] = a[r][cb];
          if (r < cb || (r == cb && ty < kk)) yc[i] = z[r][cb];
        }
        if (ty == kk) {
          const double piv = a[cb][cb];
          zp = zp || piv == 0.0;
          dinv[k] = 1.0 / piv;
        }
      }
      if (ty == kk) {
#pragma unroll
        for (int c = 0; c < LI_R; ++c) {
          const int j = tx + LI_G * c;
          if (c > cb || (c == cb && tx > kk)) row[j] = a[cb][c];
          if (c < cb || (c == cb && tx < kk)) xr[j] = z[cb][c];
        }
      }
      __syncthreads();
      const double rinv = dinv[k];
      double l[LI_R], yk[LI_R], u[LI_R], ub[LI_R], xk[LI_R];
#pragma unroll
      for (int r = 0; r < LI_R; ++r) {
        const int i = ty + LI_G * r;
        if (r > cb) {
          l[r] = col[i] * rinv;
          yk[r] = 0.0;
        } else if (r < cb) {
          l[r] = 0.0;
          yk[r] = yc[i];
        } else {
          const double cv = col[i], yv = yc[i];
          l[r] = ty > kk ? cv * rinv : 0.0;
          yk[r] = ty < kk ? yv : (ty == kk ? 1.0 : 0.0);
        }
      }
#pragma unroll
      for (int c = 0; c < LI_R; ++c) {
        const int j = tx + LI_G * c;
        if (c > cb) {
          u[c] = row[j];
          xk[c] = 0.0;
        } else if (c < cb) {
          u[c] = 0.0;
          xk[c] = xr[j];
        } else {
          const double rv = row[j], xv = xr[j];
          u[c] = tx > kk ? rv : 0.0;
          xk[c] = tx < kk ? xv : (tx == kk ? 1.0 : 0.0);
        }
        ub[c] = u[c] * rinv;
      }
      // register block (r, c) holds rows ty + 32 r, columns tx + 32 c: rows
      // of blocks r < cb and columns of blocks c < cb are <= k, those of
      // blocks > cb are > k, so the zero products drop out at compile time
#pragma unroll
      for (int r = 0; r < LI_R; ++r)
#pragma unroll
        for (int c = 0; c < LI_R; ++c) {
          if (r >= cb && c >= cb) a[r][c] -= l[r] * u[c];
          if (r >= cb && c <= cb) z[r][c] -= l[r] * xk[c];   // X: rows > k, columns <= k
          if (r <= cb && c >= cb) z[r][c] -= yk[r] * ub[c];  // Y: rows <= k, columns > k
        }
    }
  }
  if (tid >= n && tid < LUINV_N) dinv[tid] = 1.0;   // identity padding
  __syncthreads();

  // L^{-1}: strictly lower part of z, unit diagonal
#pragma unroll
  for (int r = 0; r < LI_R; ++r)
#pragma unroll
    for (int c = 0; c < LI_R; ++c) {
      const int i = ty + LI_G * r, j = tx + LI_G * c;
      stage[i + LI_S * j] = i > j ? z[r][c] : (i == j ? 1.0 : 0.0);
    }
  __syncthreads();
  for (int e = tid; e < LUINV_N * LUINV_N; e += LI_T) {
    const int i = e % LUINV_N, j = e / LUINV_N;
    if (i >= n || j >= n) continue;
    const double v = stage[i + LI_S * j];
    if (i < m1) {
      if (j < m1) it.L11[i + m1 * j] = v;
    } else {
      if (j < m1)
        it.L21[(i - m1) + m2 * j] = v;
      else
        it.L22[(i - m1) + m2 * (j - m1)] = v;
    }
  }
  __syncthreads();
  // U^{-1} = Y D^{-1}: strictly upper part of z, column j scaled by 1 / U[j, j]
#pragma unroll
  for (int r = 0; r < LI_R; ++r)
#pragma unroll
    for (int c = 0; c < LI_R; ++c) {
      const int i = ty + LI_G * r, j = tx + LI_G * c;
      const double dj = dinv[j];
      stage[i + LI_S * j] = i < j ? z[r][c] * dj : (i == j ? dj : 0.0);
    }
  __syncthreads();
  for (int e = tid; e < LUINV_N * LUINV_N; e += LI_T) {
    const int i = e % LUINV_N, j = e / LUINV_N;
    if (i >= n || j >= n) continue;
    const double v = stage[i + LI_S * j];
    if (j < m1) {
      if (i < m1) it.U11[i + m1 * j] = v;
    } else {
      if (i < m1)
        it.U12[i + m1 * (j - m1)] = v;
      else
        it.U22[(i - m1) + m2 * (j - m1)] = v;
    }
  }
  if (zp) atomicAdd(zero_pivot, 1);   // the owner of a zero pivot
}

// ---------------------------------------------------------------------------
// H-block times multi-vector: projections of the low-rank leaves, then
// owner-computes gather per output leaf cluster (no atomics, fixed order).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(HL_BLOCK) k_apply_proj(const ApplyJob* jobs, const ProjItem* items) {
  const ProjItem it = items[blockIdx.x];
  const ApplyJob J = jobs[it.job];
  const LeafDesc d = J.L[it.leaf];
  const int k = J.rank[it.leaf];
  const int kx = J.kx ? *J.kx : J.kxcap;
  double* Tl = J.T + (size_t)(it.leaf - J.lbeg) * J.tstride;
  const int len = J.trans ? d.m : d.n;
  const double* F = J.trans ? d.A : d.B;          // U (trans) or V
  const double* X = J.X + (J.trans ? (d.rlo - J.rlo) : (d.clo - J.clo));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int o = w; o < k * kx; o += 4) {
    int p = o % k, q = o / k;
    double s = 0.0;
    for (int j = lane; j < len; j += 64) s += F[j + (size_t)len * p] * X[j + (size_t)J.ldx * q];
    s = warp_sum(s);
    if (lane == 0) Tl[p + d.kcap * q] = s;
  }
}

__global__ void __launch_bounds__(HL_BLOCK) k_apply_gather(const ApplyJob* jobs, const GatherItem* items) {
  __shared__ double Xs[64 * KMAX];
  const GatherItem it = items[blockIdx.x];
  const ApplyJob J = jobs[it.job];
  const DevLists& dl = J.dl;
  const int lo = dl.lc_lo[it.lpos], hi = dl.lc_hi[it.lpos];
  const int mr = hi - lo;
  const int kx = J.kx ? *J.kx : J.kxcap;
  const int i = threadIdx.x & 63, qg = threadIdx.x >> 6;
  double acc[KMAX / 4];
  for (int u = 0; u < KMAX / 4; ++u) acc[u] = 0.0;
  const int32_t* ptr = J.trans ? dl.colptr : dl.rowptr;
  const int32_t* idx = J.trans ? dl.colidx : dl.rowidx;
  for (int e = ptr[it.lpos]; e < ptr[it.lpos + 1]; ++e) {
    const int l = idx[e];
    if (l < J.lbeg || l >= J.lend) continue;
    const LeafDesc d = J.L[l];
    if (d.kind == K_ZERO) continue;
    if (d.kind == K_DENSE) {
      const int len = J.trans ? d.m : d.n;
      const double* X = J.X + (J.trans ? (d.rlo - J.rlo) : (d.clo - J.clo));
      __syncthreads();
      for (int e2 = threadIdx.x; e2 < len * kx; e2 += HL_BLOCK)
        Xs[e2] = X[(e2 % len) + (size_t)J.ldx * (e2 / len)];
      __syncthreads();
      if (i < mr) {
        // row i of the block in 16-column chunks, each chunk loaded once
        // and applied to every column q = qg + 4 u of X (wavefront-uniform
        // guards keep the accumulator indices static)
        const double* D = J.trans ? d.A + (size_t)d.m * (lo - d.clo) : d.A + (lo - d.rlo);
        const size_t si = J.trans ? (size_t)d.m : 1, sj = J.trans ? 1 : (size_t)d.m;
        for (int j0 = 0; j0 < len; j0 += 16) {
          const int jn = min(16, len - j0);
          double dv[16];
#pragma unroll
          for (int jj = 0; jj < 16; ++jj) dv[jj] = jj < jn ? D[si * i + sj * (j0 + jj)] : 0.0;
#pragma unroll
          for (int u = 0; u < KMAX / 4; ++u) {
            if (qg + 4 * u >= kx) break;
            const double* xq = Xs + len * (qg + 4 * u) + j0;
            double s = 0.0;
#pragma unroll
            for (int jj = 0; jj < 16; ++jj) s += dv[jj] * (jj < jn ? xq[jj] : 0.0);
            acc[u] += s;
          }
        }
      }
    } else {
      const int k = J.rank[l];
      const double* Tl = J.T + (size_t)(l - J.lbeg) * J.tstride;
      if (i < mr) {
        // row i of the factor loaded once, applied to every column q
        const double* F = J.trans ? d.B + (lo - d.clo) : d.A + (lo - d.rlo);
        const int ld = J.trans ? d.n : d.m;
        for (int p0 = 0; p0 < k; p0 += 16) {
          const int pn = min(16, k - p0);
          double fv[16];
#pragma unroll
          for (int pp = 0; pp < 16; ++pp) fv[pp] = pp < pn ? F[i + (size_t)ld * (p0 + pp)] : 0.0;
#pragma unroll
          for (int u = 0; u < KMAX / 4; ++u) {
            if (qg + 4 * u >= kx) break;
            const double* tq = Tl + d.kcap * (qg + 4 * u) + p0;
            double s = 0.0;
#pragma unroll
            for (int pp = 0; pp < 16; ++pp) s += fv[pp] * (pp < pn ? tq[pp] : 0.0);
            acc[u] += s;
          }
        }
      }
    }
  }
  if (i < mr) {
    double* Y = J.Y + (lo - (J.trans ? J.clo : J.rlo));
    for (int u = 0; qg + 4 * u < kx; ++u) Y[i + (size_t)J.ldy * (qg + 4 * u)] = acc[u];
  }
}

// ---------------------------------------------------------------------------
// vectors: permutation, Crank-Nicolson right-hand side, refinement
// ---------------------------------------------------------------------------
__global__ void k_perm_gather(double* out, const double* in, const int32_t* perm, int N) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) out[i] = in[perm[i]];
}
__global__ void k_perm_scatter(double* out, const double* in, const int32_t* perm, int N) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) out[perm[i]] = in[i];
}
// out = x + a*y (+ cg * g if g)
__global__ void k_axpy2(double* out, const double* x, double a, const double* y, double cg,
                        const double* g, int N) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) {
    double v = x[i] + a * y[i];
    if (g) v += cg * g[i];
    out[i] = v;
  }
}
// r = b - (x - hdt * Gx)
__global__ void k_residual(double* r, const double* b, const double* x, const double* Gx, double hdt, int N) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) r[i] = b[i] - (x[i] - hdt * Gx[i]);
}
__global__ void k_add(double* x, const double* d, int N) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) x[i] += d[i];
}
// deterministic two-level sum of squares: partial[b] per block, then one block
__global__ void __launch_bounds__(HL_BLOCK) k_sumsq_partial(const double* x, int N, double* partial) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = blockIdx.x * HL_BLOCK + threadIdx.x; i < N; i += gridDim.x * HL_BLOCK) s += x[i] * x[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
__global__ void __launch_bounds__(HL_BLOCK) k_sum_final(const double* partial, int n, double* out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += HL_BLOCK) s += partial[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s;
}

// Residual check of a refinement: partial[2 b] = sum of r_i^2 and
// partial[2 b + 1] = sum of (alpha u_i + cg g_i)^2 over block b's slice (the
// right-hand side of the system whose residual r is; g may be null), then
// one block adds the partials in a fixed order into out[0], out[1]
// (deterministic: the grid depends on N only).
__global__ void __launch_bounds__(HL_BLOCK) k_check_partial(const double* r, const double* u, double alpha,
                                                            const double* g, double cg, int N, double* partial) {
  __shared__ double red[4];
  double sr = 0.0, sb = 0.0;
  for (int i = blockIdx.x * HL_BLOCK + threadIdx.x; i < N; i += gridDim.x * HL_BLOCK) {
    const double b = alpha * u[i] + (g ? cg * g[i] : 0.0);
    sr += r[i] * r[i];
    sb += b * b;
  }
  sr = block_sum(sr, red);
  sb = block_sum(sb, red);
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = sr;
    partial[2 * blockIdx.x + 1] = sb;
  }
}
__global__ void __launch_bounds__(HL_BLOCK) k_check_final(const double* partial, int n, double* out) {
  __shared__ double red[4];
  double sr = 0.0, sb = 0.0;
  for (int i = threadIdx.x; i < n; i += HL_BLOCK) {
    sr += partial[2 * i];
    sb += partial[2 * i + 1];
  }
  sr = block_sum(sr, red);
  sb = block_sum(sb, red);
  if (threadIdx.x == 0) {
    out[0] = sr;
    out[1] = sb;
  }
}
// u = w - u  (Crank-Nicolson: u^{n+1} = w - u^n)
__global__ void k_wsub(double* u, const double* w, int N) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < N) u[i] = w[i] - u[i];
}

// densify: every leaf writes its block into the natural-order dense matrix
__global__ void __launch_bounds__(HL_BLOCK) k_densify(const LeafDesc* L, const int32_t* rank,
                                                      const int32_t* perm, int N, double* dense) {
  const LeafDesc d = L[blockIdx.x];
  const int k = d.kind == K_LR ? rank[blockIdx.x] : 0;
  for (int e = threadIdx.x; e < d.m * d.n; e += HL_BLOCK) {
    int i = e % d.m, j = e / d.m;
    double v = 0.0;
    if (d.kind == K_DENSE) v = d.A[e];
    else if (d.kind == K_LR)
      for (int p = 0; p < k; ++p) v += d.A[i + (size_t)d.m * p] * d.B[j + (size_t)d.n * p];
    dense[(size_t)perm[d.rlo + i] * N + perm[d.clo + j]] = v;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline hipError_t post() { return hipGetLastError(); }

hipError_t launch_constants_var(const ProblemDev& P, double* out, hipStream_t s) {
  if (P.nvar < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_constants_var, dim3(P.nvar), dim3(HL_BLOCK), 0, s, P, out);
  return post();
}

hipError_t launch_constants(const ProblemDev& P, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_constants, dim3(1), dim3(HL_BLOCK), 0, s, P, out);
  return post();
}
hipError_t launch_fill_dense(const ProblemDev& P, const double* cst, const int32_t* perm,
                             const LeafDesc* L, const int32_t* ids, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_dense, dim3(n), dim3(HL_BLOCK), 0, s, P, cst, perm, L, ids);
  return post();
}
hipError_t launch_exterior(const ProblemDev& P, const double* cst, const double* u_ext, double* tab, double* g,
                           hipStream_t s) {
  const int NW = P.n + 1;
  hipLaunchKernelGGL(k_ext_table, dim3((2 * NW + 1 + HL_BLOCK - 1) / HL_BLOCK), dim3(HL_BLOCK), 0, s, P, cst, tab);
  hipLaunchKernelGGL(k_ext_apply, dim3(P.n), dim3(HL_BLOCK), 0, s, tab, u_ext, P.n, g);
  return post();
}
hipError_t launch_exterior2(const ProblemDev& P, const double* cst, const double* u_ext, int ld, int org,
                            double* tab, double* g, hipStream_t s) {
  const long side = 2 * (long)(P.n + 1) + 1;
  hipLaunchKernelGGL(k_ext2_table, dim3((unsigned)((side * side + HL_BLOCK - 1) / HL_BLOCK)), dim3(HL_BLOCK), 0, s,
                     P, cst, tab);
  hipLaunchKernelGGL(k_ext2_apply, dim3(P.n * P.n), dim3(HL_BLOCK), 0, s, tab, u_ext, P.n, ld, org, g);
  return post();
}
hipError_t launch_far_field2(const ProblemDev& P, const double* u_ext, int next, double tail_left,
                             double tail_right, double* tab, double* g, hipStream_t s) {
  const long side = 2 * (long)next + 1;
  double* tails = tab + side * side;
  hipLaunchKernelGGL(k_far2_table, dim3((unsigned)((side * side + HL_BLOCK - 1) / HL_BLOCK)), dim3(HL_BLOCK), 0, s,
                     P, next, tab);
  hipLaunchKernelGGL(k_far2_tails, dim3(1), dim3(32), 0, s, P, next * P.h, tails);
  hipLaunchKernelGGL(k_far2_apply, dim3(P.n * P.n), dim3(HL_BLOCK), 0, s, tab, tails, u_ext, P.n, next, tail_left,
                     tail_right, g);
  return post();
}
hipError_t launch_far_field(const ProblemDev& P, const double* u_ext, int next, double tail_left,
                            double tail_right, double* tab, double* g, hipStream_t s) {
  const int cnt = next - (P.n + 1) + 1;
  hipLaunchKernelGGL(k_far_table, dim3((cnt + HL_BLOCK - 1) / HL_BLOCK), dim3(HL_BLOCK), 0, s, P, next, tab);
  hipLaunchKernelGGL(k_far_apply, dim3(P.n), dim3(HL_BLOCK), 0, s, tab, u_ext, P.n, next, tail_left, tail_right, g);
  return post();
}
hipError_t launch_taylor(const ProblemDev& P, const int32_t* perm, const LeafDesc* L, const int32_t* ids, int n,
                         int32_t* rank, int r, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_taylor, dim3(n), dim3(HL_BLOCK), 0, s, P, perm, L, ids, rank, r);
  return post();
}
hipError_t launch_aca(const ProblemDev& P, const int32_t* perm, const LeafDesc* L, const int32_t* ids,
                      int n, double* U, double* V, const int64_t* uoff, const int64_t* voff,
                      int32_t* ranks, int kcap, double eps, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_aca, dim3(n), dim3(HL_BLOCK), 0, s, P, perm, L, ids, U, V, uoff, voff, ranks,
                     kcap, eps);
  return post();
}
hipError_t launch_flush_lr(const LFlushTarget* tg, int ntg, const Term* terms, const ChunkItem* gram,
                           int ngram, const ChunkItem* expand, int nexp, double tol, int ks, hipStream_t s) {
  if (ntg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_flush_gram, dim3(ngram), dim3(HL_BLOCK), 0, s, tg, terms, gram, tol);
  // the pivoted-Cholesky core: up to 48 columns with double-double parts,
  // up to KMAX without (tolerances >= RADD_DD_TOL)
  if (ks <= 48 || (!radd_needs_dd(tol) && ks <= KMAX)) {
    hipLaunchKernelGGL(k_flush_core_fast, dim3(ntg), dim3(HL_BLOCK), radd_core_lds(ks, radd_needs_dd(tol)), s, tg,
                       terms, tol, ks);
  } else {
    size_t shm = (4 * (size_t)ks * ks + 2 * (size_t)ks) * sizeof(double);
    hipLaunchKernelGGL(k_flush_core, dim3(ntg), dim3(HL_BLOCK), shm, s, tg, terms, tol, ks);
  }
  hipLaunchKernelGGL(k_flush_expand, dim3(nexp), dim3(HL_BLOCK), 0, s, tg, terms, expand);
  return post();
}
static size_t radd_fused_dyn_lds(int k, double tol) {
  return std::max(radd_fused_lds(k, radd_needs_dd(tol)), (size_t)2 * DF_KC * 64 * sizeof(double));
}
hipError_t launch_radd_fused(const LFlushTarget* tg, int ntg, const Term* terms, double tol, int ks, hipStream_t s,
                             const DFlushItem* dflush, int ndflush, const Term* dterms) {
  if (ntg == 0 && ndflush == 0) return hipSuccess;
  if (ks > fused_width(tol)) return hipErrorInvalidValue;
  const int k = ks < 32 ? 32 : ks;
  hipLaunchKernelGGL(k_radd_fused, dim3(ntg + ndflush), dim3(HL_BLOCK), radd_fused_dyn_lds(k, tol), s, tg, ntg,
                     terms, tol, k, dflush, dterms);
  return post();
}
hipError_t launch_flush_dense(const DFlushItem* items, int n, const Term* terms, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_flush_dense, dim3(n), dim3(HL_BLOCK), 0, s, items, terms);
  return post();
}
hipError_t launch_dense_prod(const DProdItem* items, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_dense_prod, dim3(n), dim3(HL_BLOCK), 0, s, items);
  return post();
}
hipError_t launch_copy(const CopyItem* items, int n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_leaf, dim3(n), dim3(HL_BLOCK), 0, s, items);
  return post();
}
hipError_t launch_lu_inv(const LuInvItem* items, int n, int32_t* zero_pivot, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lu_inv, dim3(n), dim3(LI_T), luinv_lds_bytes(), s, items, zero_pivot);
  return post();
}
hipError_t launch_getrf_inv(const GetrfItem* items, int n, int32_t* zero_pivot, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_getrf_inv, dim3(n), dim3(HL_BLOCK), 0, s, items, zero_pivot);
  return post();
}
hipError_t launch_apply(const ApplyJob* jobs, const ProjItem* proj, int nproj, const GatherItem* gat,
                        int ngat, hipStream_t s) {
  if (nproj > 0) hipLaunchKernelGGL(k_apply_proj, dim3(nproj), dim3(HL_BLOCK), 0, s, jobs, proj);
  if (ngat > 0) hipLaunchKernelGGL(k_apply_gather, dim3(ngat), dim3(HL_BLOCK), 0, s, jobs, gat);
  return post();
}
static inline dim3 grid1(int N) { return dim3((N + HL_BLOCK - 1) / HL_BLOCK); }
hipError_t launch_perm_gather(double* out, const double* in, const int32_t* perm, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_gather, grid1(N), dim3(HL_BLOCK), 0, s, out, in, perm, N);
  return post();
}
hipError_t launch_perm_scatter(double* out, const double* in, const int32_t* perm, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_scatter, grid1(N), dim3(HL_BLOCK), 0, s, out, in, perm, N);
  return post();
}
hipError_t launch_axpy2(double* out, const double* x, double a, const double* y, double cg,
                        const double* g, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy2, grid1(N), dim3(HL_BLOCK), 0, s, out, x, a, y, cg, g, N);
  return post();
}
hipError_t launch_residual(double* r, const double* b, const double* x, const double* Gx, double hdt,
                           int N, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, grid1(N), dim3(HL_BLOCK), 0, s, r, b, x, Gx, hdt, N);
  return post();
}
hipError_t launch_add(double* x, const double* d, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_add, grid1(N), dim3(HL_BLOCK), 0, s, x, d, N);
  return post();
}
hipError_t launch_sumsq(const double* x, int N, double* partial, int nblocks, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sumsq_partial, dim3(nblocks), dim3(HL_BLOCK), 0, s, x, N, partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(HL_BLOCK), 0, s, partial, nblocks, out);
  return post();
}
int check_blocks(int N) { return std::max(1, std::min(256, (N + 1023) / 1024)); }
hipError_t launch_check_norms(const double* r, const double* u, double alpha, const double* g, double cg, int N,
                              double* partial, double* out, hipStream_t s) {
  const int nb = check_blocks(N);
  hipLaunchKernelGGL(k_check_partial, dim3(nb), dim3(HL_BLOCK), 0, s, r, u, alpha, g, cg, N, partial);
  hipLaunchKernelGGL(k_check_final, dim3(1), dim3(HL_BLOCK), 0, s, partial, nb, out);
  return post();
}
hipError_t launch_wsub(double* u, const double* w, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_wsub, grid1(N), dim3(HL_BLOCK), 0, s, u, w, N);
  return post();
}
hipError_t launch_densify(const LeafDesc* L, const int32_t* rank, int nleaves, const int32_t* perm,
                          int N, double* dense, hipStream_t s) {
  hipLaunchKernelGGL(k_densify, dim3(nleaves), dim3(HL_BLOCK), 0, s, L, rank, perm, N, dense);
  return post();
}

}  // namespace hl

namespace hl {
hipError_t init_kernel_attributes() {
  hipError_t e = hipFuncSetAttribute((const void*)k_flush_core_fast, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)radd_core_lds(48));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_radd_fused, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)radd_fused_lds(48));
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)k_lu_inv, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)luinv_lds_bytes());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_flush_core, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (4 * KMAX * KMAX + 2 * KMAX) * (int)sizeof(double));
}
}  // namespace hl
