// HIP kernels for gfx950 (CDNA4, 64-wide wavefronts) of the H-matrix
// Crank-Nicolson library.  Host-side launchers are at the end of the file.
#include <hip/hip_runtime.h>

#include <cmath>

#include "hl_jobs.h"
#include "hl_kernels.h"

namespace hl {

#define HL_BLOCK 256

// ---------------------------------------------------------------------------
// double-double helpers (error-free transformations; FMA for products)
// ---------------------------------------------------------------------------
struct dd {
  double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
__device__ __forceinline__ dd quick_two_sum(double a, double b) {
  double s = a + b;
  return {s, b - (s - a)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = quick_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return quick_two_sum(s.hi, s.lo);
}
__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  double p = a.hi * b.hi;
  double e = fma(a.hi, b.hi, -p);
  e += a.hi * b.lo + a.lo * b.hi;
  return quick_two_sum(p, e);
}
__device__ __forceinline__ dd dd_mul_d(double a, double b) {
  double p = a * b;
  return {p, fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_div(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd r = dd_add(a, dd_neg(dd_mul({q1, 0.0}, b)));
  double q2 = r.hi / b.hi;
  r = dd_add(r, dd_neg(dd_mul({q2, 0.0}, b)));
  double q3 = r.hi / b.hi;
  dd q = quick_two_sum(q1, q2);
  return dd_add(q, {q3, 0.0});
}
__device__ __forceinline__ dd dd_sqrt(dd a) {
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

// ---------------------------------------------------------------------------
// kernel of the jump measure and quadrature constants (Sec. 4)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double nu_at(const ProblemDev& P, double r) {
  return P.C * exp(-P.lam * r) / pow(r, (double)P.dim + 2.0 * P.s);
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

// upper incomplete gamma Gamma(a, x) for a in (-2, 1], x > 0
__device__ double upper_gamma(double a, double x) {
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

// out = {S0, S2, C2, T}.  One block.
//   S0 = sum' W_k nu(kh) over the window |k|_inf <= NW = n + 1 (L_W = (n+1)h),
//        trapezoid weights h (h/2 on the window edge) per axis;
//   S2 = sum' W_k rho_k nu(kh) (k_1 h)^2 with rho the grid window of radius
//        m = round(r0/h) (weight 1/2 on its edge);
//   C2 = int rho nu y_1^2 dy,  T = int_{|y|_inf > L_W} nu dy.
__global__ void __launch_bounds__(HL_BLOCK) k_constants(ProblemDev P, double* out) {
  __shared__ double red[4];
  __shared__ double glx[32], glw[32];
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
  if (P.dim == 1) {
    for (int k = 1 + threadIdx.x; k <= NW; k += blockDim.x) {
      double w = (k == NW) ? 0.5 * h : h;
      double nu = nu_at(P, k * h);
      acc(s0, s0c, 2.0 * w * nu);
      if (k <= m) {
        double rho = (k < m) ? 1.0 : 0.5;
        acc(s2, s2c, 2.0 * w * rho * nu * (k * h) * (k * h));
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
      double nu = nu_at(P, rr);
      acc(s0, s0c, w * nu);
      if (abs(k1) <= m && abs(k2) <= m) {
        double rho = ((abs(k1) < m) ? 1.0 : 0.5) * ((abs(k2) < m) ? 1.0 : 0.5);
        acc(s2, s2c, w * rho * nu * (k1 * h) * (k1 * h));
      }
    }
  }
  double S0 = block_sum(s0, red) + block_sum(s0c, red);
  double S2 = block_sum(s2, red) + block_sum(s2c, red);
  if (threadIdx.x < 32) gauss_legendre(32, threadIdx.x, &glx[threadIdx.x], &glw[threadIdx.x]);
  __syncthreads();
  if (threadIdx.x == 0) {
    const double s = P.s, C = P.C, lam = P.lam, a2 = 2.0 - 2.0 * s;
    double C2 = 0.0, T = 0.0;
    if (P.dim == 1) {
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
  }
}

// Generator entry G_ij (cluster-ordered i, j) from integer grid offsets.
__device__ __forceinline__ double gen_entry(const ProblemDev& P, const double* cst,
                                            const int32_t* perm, int i, int j) {
  const double h = P.h;
  const double beta = 0.5 * (cst[2] - cst[1]);
  int k1, k2 = 0;
  if (P.dim == 1) {
    k1 = j - i;
  } else {
    int pi = perm[i], pj = perm[j];
    k1 = pj / P.n - pi / P.n;
    k2 = pj % P.n - pi % P.n;
  }
  if (k1 == 0 && k2 == 0)
    return -cst[0] - cst[3] - 2.0 * P.dim * (beta + P.a) / (h * h) + P.c;
  double rr = h * sqrt((double)k1 * k1 + (double)k2 * k2);
  double v = (P.dim == 1 ? h : h * h) * nu_at(P, rr);
  if (abs(k1) + abs(k2) == 1) {
    v += (beta + P.a) / (h * h);
    if (k1 != 0) v += (k1 > 0 ? 1.0 : -1.0) * P.b0 / (2.0 * h);
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
  double rr = P.h * sqrt((double)k1 * k1 + (double)k2 * k2);
  return (P.dim == 1 ? P.h : P.h * P.h) * nu_at(P, rr);
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
  __shared__ uint32_t used[512];   // up to 16384 rows
  const LeafDesc d = L[ids[blockIdx.x]];
  double* U = Ubuf + uoff[blockIdx.x];
  double* V = Vbuf + voff[blockIdx.x];
  const int m = d.m, n = d.n;
  const int kmax = min(kcap, min(m, n));
  for (int q = threadIdx.x; q < 512; q += blockDim.x) used[q] = 0u;
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
struct ColMap {
  int K, kC, nt;
  int off[KMAX + 1];
  int kt[KMAX];
};

__device__ void build_colmap(const LFlushTarget& T, const Term* terms, int kC, ColMap& cm) {
  cm.kC = kC;
  cm.nt = T.tcount;
  int K = kC;
  for (int t = 0; t < T.tcount; ++t) {
    const Term& tm = terms[T.tbeg + t];
    int kt = tm.k ? *tm.k : tm.kfix;
    cm.off[t] = K;
    cm.kt[t] = kt;
    K += kt;
  }
  cm.off[T.tcount] = K;
  cm.K = K;
}

// value of column j of the concatenated factor on side 0 (U side) or 1 (V side)
__device__ __forceinline__ double side_val(const LFlushTarget& T, const Term* terms, const ColMap& cm,
                                           int side, int row, int j) {
  if (j < cm.kC) return side == 0 ? T.U[row + (size_t)T.m * j] : T.V[row + (size_t)T.n * j];
  int t = 0;
  while (j >= cm.off[t + 1]) ++t;
  const Term& tm = terms[T.tbeg + t];
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

// partial Gram of rows [r0, r1) of one side, double-double, packed upper triangle
__global__ void __launch_bounds__(HL_BLOCK) k_flush_gram(const LFlushTarget* tg, const Term* terms,
                                                         const ChunkItem* items) {
  __shared__ ColMap cm;
  __shared__ double tile[64 * KMAX];
  const ChunkItem it = items[blockIdx.x];
  const LFlushTarget T = tg[it.tgt];
  if (threadIdx.x == 0) build_colmap(T, terms, T.rank ? *T.rank : 0, cm);
  __syncthreads();
  const int K = cm.K;
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
    int rows = min(64, it.r1 - base);
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * K; e += HL_BLOCK) {
      int rr = e % 64, j = e / 64;
      tile[rr + 64 * j] = rr < rows ? side_val(T, terms, cm, it.side, base + rr, j) : 0.0;
    }
    __syncthreads();
    for (int u = 0; u < PPT; ++u) {
      if (pp[u] < 0) continue;
      const double* a = tile + 64 * pp[u];
      const double* b = tile + 64 * qq[u];
      dd s = accv[u];
      for (int rr = 0; rr < rows; ++rr) s = dd_add(s, dd_mul_d(a[rr], b[rr]));
      accv[u] = s;
    }
  }
  const int Kc = T.Kcap;
  double* dst = T.ws + (size_t)(it.side == 0 ? it.chunk : T.nchA + it.chunk) * npairs(Kc) * 2;
  for (int u = 0; u < PPT; ++u) {
    if (pp[u] < 0) continue;
    int idx = pair_index(pp[u], qq[u]);
    dst[2 * idx] = accv[u].hi;
    dst[2 * idx + 1] = accv[u].lo;
  }
}

// pivoted Cholesky (double-double) of the Gram G (K x K, full, in Gh/Gl);
// writes R (rank x K, original column order, row-major stride KMAX) and
// returns the rank.
__device__ int pivoted_cholesky(double* Gh, double* Gl, double* R, int K, int* sel, double* rowh,
                                double* rowl, int* shared_int, double* shared_d) {
  const int tid = threadIdx.x;
  for (int e = tid; e < KMAX * KMAX; e += HL_BLOCK) R[e] = 0.0;
  if (tid < KMAX) sel[tid] = 0;
  if (tid == 0) {
    double mx = 0.0;
    for (int p = 0; p < K; ++p) mx = fmax(mx, Gh[p * KMAX + p]);
    shared_d[0] = mx;
  }
  __syncthreads();
  const double dmax0 = shared_d[0];
  int r = 0;
  for (int j = 0; j < K; ++j) {
    if (tid == 0) {
      int best = -1;
      dd bv = {-1.0, 0.0};
      for (int p = 0; p < K; ++p) {
        if (sel[p]) continue;
        dd v = {Gh[p * KMAX + p], Gl[p * KMAX + p]};
        if (v.hi > bv.hi || (v.hi == bv.hi && v.lo > bv.lo)) { bv = v; best = p; }
      }
      if (best < 0 || !(bv.hi > 1e-32 * dmax0) || !(bv.hi > 0.0)) best = -1;
      shared_int[0] = best;
      if (best >= 0) sel[best] = 1;
    }
    __syncthreads();
    const int p = shared_int[0];
    if (p < 0) break;
    const dd rjj = dd_sqrt({Gh[p * KMAX + p], Gl[p * KMAX + p]});
    for (int q = tid; q < K; q += HL_BLOCK) {
      dd v;
      if (q == p) v = rjj;
      else if (sel[q]) v = {0.0, 0.0};
      else v = dd_div({Gh[p * KMAX + q], Gl[p * KMAX + q]}, rjj);
      rowh[q] = v.hi;
      rowl[q] = v.lo;
      R[j * KMAX + q] = v.hi + v.lo;
    }
    __syncthreads();
    for (int e = tid; e < K * K; e += HL_BLOCK) {
      int q1 = e / K, q2 = e % K;
      if (sel[q1] || sel[q2]) continue;
      dd g = {Gh[q1 * KMAX + q2], Gl[q1 * KMAX + q2]};
      g = dd_add(g, dd_neg(dd_mul({rowh[q1], rowl[q1]}, {rowh[q2], rowl[q2]})));
      Gh[q1 * KMAX + q2] = g.hi;
      Gl[q1 * KMAX + q2] = g.lo;
    }
    __syncthreads();
    r = j + 1;
  }
  __syncthreads();
  return r;
}

// One block per target: Gram sums -> R_A, R_B -> M = R_A R_B^T -> one-sided
// Jacobi SVD -> truncation (relative Frobenius tol) -> Y_U = R_B^T Z_r and
// Y_V = R_A^T W_r Sigma_r^{-1}, so that U_new = A Y_U and V_new = B Y_V.
__global__ void __launch_bounds__(HL_BLOCK) k_flush_core(const LFlushTarget* tg, const Term* terms,
                                                         double tol) {
  extern __shared__ double smem[];
  double* Gh = smem;                     // KMAX*KMAX
  double* Gl = Gh + KMAX * KMAX;         // KMAX*KMAX
  double* RA = Gl + KMAX * KMAX;         // KMAX*KMAX
  double* RB = RA + KMAX * KMAX;         // KMAX*KMAX
  __shared__ ColMap cm;
  __shared__ int sel[KMAX];
  __shared__ double rowh[KMAX], rowl[KMAX];
  __shared__ int sint[4];
  __shared__ double sdbl[4];
  __shared__ double sig[KMAX];
  __shared__ int order[KMAX];
  __shared__ int rot_count;
  const LFlushTarget T = tg[blockIdx.x];
  const int tid = threadIdx.x;
  const int kC = T.rank ? *T.rank : 0;
  if (tid == 0) build_colmap(T, terms, kC, cm);
  __syncthreads();
  const int K = cm.K;
  const int Kc = T.Kcap;
  const int np = npairs(Kc);
  int rk[2];
  for (int side = 0; side < 2; ++side) {
    const int nch = side == 0 ? T.nchA : T.nchB;
    const double* src = T.ws + (size_t)(side == 0 ? 0 : T.nchA) * np * 2;
    for (int e = tid; e < K * K; e += HL_BLOCK) {
      int p = e / K, q = e % K;
      int a = min(p, q), b = max(p, q);
      int idx = pair_index(a, b);
      dd s = {0.0, 0.0};
      for (int c = 0; c < nch; ++c) s = dd_add(s, {src[(size_t)c * np * 2 + 2 * idx], src[(size_t)c * np * 2 + 2 * idx + 1]});
      Gh[p * KMAX + q] = s.hi;
      Gl[p * KMAX + q] = s.lo;
    }
    __syncthreads();
    rk[side] = pivoted_cholesky(Gh, Gl, side == 0 ? RA : RB, K, sel, rowh, rowl, sint, sdbl);
    __syncthreads();
  }
  const int rA = rk[0], rB = rk[1];
  // M (rA x rB) column-major with stride KMAX, Z (rB x rB)
  double* M = Gh;
  double* Z = Gl;
  for (int e = tid; e < KMAX * KMAX; e += HL_BLOCK) { M[e] = 0.0; Z[e] = 0.0; }
  __syncthreads();
  for (int e = tid; e < rA * rB; e += HL_BLOCK) {
    int i = e % rA, j = e / rA;
    double s = 0.0;
    for (int q = 0; q < K; ++q) s += RA[i * KMAX + q] * RB[j * KMAX + q];
    M[i + KMAX * j] = s;
  }
  for (int e = tid; e < rB; e += HL_BLOCK) Z[e + KMAX * e] = 1.0;
  __syncthreads();
  // one-sided Jacobi on the columns of M; disjoint pairs per round
  const int nn = rB + (rB & 1);
  const int g = tid >> 3, l8 = tid & 7;
  for (int sweep = 0; sweep < 60 && nn >= 2; ++sweep) {
    if (tid == 0) rot_count = 0;
    __syncthreads();
    for (int rd = 0; rd < nn - 1; ++rd) {
      if (g < nn / 2) {
        int a = (rd + g) % (nn - 1);
        int b = (g == 0) ? nn - 1 : (rd - g + nn - 1) % (nn - 1);
        if (a > b) { int t = a; a = b; b = t; }
        bool active = (b < rB);
        double al = 0.0, be = 0.0, ga = 0.0;
        if (active) {
          for (int i = l8; i < rA; i += 8) {
            double x = M[i + KMAX * a], y = M[i + KMAX * b];
            al += x * x; be += y * y; ga += x * y;
          }
        }
        for (int o = 4; o > 0; o >>= 1) {
          al += __shfl_xor(al, o, 8);
          be += __shfl_xor(be, o, 8);
          ga += __shfl_xor(ga, o, 8);
        }
        if (active && ga != 0.0 && fabs(ga) > 1e-15 * sqrt(al * be)) {
          double zeta = (be - al) / (2.0 * ga);
          double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
          for (int i = l8; i < rA; i += 8) {
            double x = M[i + KMAX * a], y = M[i + KMAX * b];
            M[i + KMAX * a] = c * x - s * y;
            M[i + KMAX * b] = s * x + c * y;
          }
          for (int i = l8; i < rB; i += 8) {
            double x = Z[i + KMAX * a], y = Z[i + KMAX * b];
            Z[i + KMAX * a] = c * x - s * y;
            Z[i + KMAX * b] = s * x + c * y;
          }
          if (l8 == 0) atomicAdd(&rot_count, 1);
        }
      }
      __syncthreads();
    }
    int rc = rot_count;
    __syncthreads();
    if (rc == 0) break;
  }
  for (int c = tid; c < rB; c += HL_BLOCK) {
    double s = 0.0;
    for (int i = 0; i < rA; ++i) s += M[i + KMAX * c] * M[i + KMAX * c];
    sig[c] = sqrt(s);
  }
  __syncthreads();
  if (tid == 0) {
    for (int c = 0; c < rB; ++c) order[c] = c;
    for (int a = 1; a < rB; ++a) {  // insertion sort, descending
      int v = order[a], b = a - 1;
      while (b >= 0 && sig[order[b]] < sig[v]) { order[b + 1] = order[b]; --b; }
      order[b + 1] = v;
    }
    double tot = 0.0;
    for (int c = 0; c < rB; ++c) tot += sig[c] * sig[c];
    int r = rB;
    double tail = 0.0;
    while (r > 0) {
      double sgm = sig[order[r - 1]];
      if (tail + sgm * sgm <= tol * tol * tot) { tail += sgm * sgm; --r; } else break;
    }
    if (!(tot > 0.0)) r = 0;
    int ovf = 0;
    if (r > T.kcap) { r = T.kcap; ovf = 1; }
    sint[0] = r;
    T.info[0] = kC;
    T.info[1] = r;
    T.info[2] = ovf;
    if (ovf && T.overflow) atomicAdd(T.overflow, 1);
    if (T.rank) *T.rank = r;
  }
  __syncthreads();
  const int r = sint[0];
  double* YU = T.ws + (size_t)(T.nchA + T.nchB) * np * 2;
  double* YV = YU + (size_t)Kc * T.kcap;
  for (int e = tid; e < K * r; e += HL_BLOCK) {
    int q = e % K, c = e / K;
    int oc = order[c];
    double su = 0.0, sv = 0.0;
    for (int i = 0; i < rB; ++i) su += RB[i * KMAX + q] * Z[i + KMAX * oc];
    for (int i = 0; i < rA; ++i) sv += RA[i * KMAX + q] * M[i + KMAX * oc];
    double sg = sig[oc];
    YU[q + (size_t)Kc * c] = su;
    YV[q + (size_t)Kc * c] = sv / (sg * sg);
  }
}

// U_new = A Y_U (side 0) or V_new = B Y_V (side 1) for rows [r0, r1)
__global__ void __launch_bounds__(HL_BLOCK) k_flush_expand(const LFlushTarget* tg, const Term* terms,
                                                           const ChunkItem* items) {
  __shared__ ColMap cm;
  __shared__ double Y[KMAX * 32];
  const ChunkItem it = items[blockIdx.x];
  const LFlushTarget T = tg[it.tgt];
  const int kC = T.info[0], r = T.info[1];
  if (threadIdx.x == 0) build_colmap(T, terms, kC, cm);
  __syncthreads();
  const int K = cm.K, Kc = T.Kcap;
  const int np = npairs(Kc);
  const double* Ys = T.ws + (size_t)(T.nchA + T.nchB) * np * 2 + (it.side == 0 ? 0 : (size_t)Kc * T.kcap);
  for (int e = threadIdx.x; e < K * r; e += HL_BLOCK) Y[e] = Ys[(e % K) + (size_t)Kc * (e / K)];
  __syncthreads();
  double* out = it.side == 0 ? T.U : T.V;
  const int ld = it.side == 0 ? T.m : T.n;
  for (int row = it.r0 + threadIdx.x; row < it.r1; row += HL_BLOCK) {
    double acc[32];
    for (int c = 0; c < 32; ++c) acc[c] = 0.0;
    for (int j = 0; j < K; ++j) {
      double a = side_val(T, terms, cm, it.side, row, j);
      for (int c = 0; c < r; ++c) acc[c] += a * Y[j + K * c];
    }
    for (int c = 0; c < r; ++c) out[row + (size_t)ld * c] = acc[c];
  }
}

// ---------------------------------------------------------------------------
// dense targets, products, copies, leaf factorisation
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(HL_BLOCK) k_flush_dense(const DFlushItem* items, const Term* terms) {
  const DFlushItem it = items[blockIdx.x];
  for (int t = 0; t < it.tcount; ++t) {
    const Term tm = terms[it.tbeg + t];
    const int k = tm.dense ? 0 : (tm.k ? *tm.k : tm.kfix);
    const int tot = tm.mr * tm.nc;
    for (int e = threadIdx.x; e < tot; e += HL_BLOCK) {
      int i = e % tm.mr, j = e / tm.mr;
      double v;
      if (tm.dense) {
        v = tm.U[i + (size_t)tm.ldu * j];
      } else {
        v = 0.0;
        for (int p = 0; p < k; ++p) v += tm.U[i + (size_t)tm.ldu * p] * tm.W[j + (size_t)tm.ldw * p];
      }
      it.D[(tm.ro + i) + (size_t)it.ldd * (tm.co + j)] += tm.sign * v;
    }
    __syncthreads();
  }
}

__global__ void __launch_bounds__(HL_BLOCK) k_dense_prod(const DProdItem* items) {
  __shared__ double As[64 * 64], Bs[64 * 64];
  const DProdItem it = items[blockIdx.x];
  for (int e = threadIdx.x; e < it.m * it.k; e += HL_BLOCK) As[e] = it.A[(e % it.m) + (size_t)it.lda * (e / it.m)];
  for (int e = threadIdx.x; e < it.k * it.n; e += HL_BLOCK) Bs[e] = it.B[(e % it.k) + (size_t)it.ldb * (e / it.k)];
  __syncthreads();
  for (int e = threadIdx.x; e < it.m * it.n; e += HL_BLOCK) {
    int i = e % it.m, j = e / it.m;
    double s = 0.0;
    for (int q = 0; q < it.k; ++q) s += As[i + it.m * q] * Bs[q + it.k * j];
    it.P[i + (size_t)it.ldp * j] = s;
  }
}

__global__ void __launch_bounds__(HL_BLOCK) k_copy_leaf(const CopyItem* items) {
  const CopyItem it = items[blockIdx.x];
  if (it.dense) {
    const int tot = it.m * it.n;
    for (int e = threadIdx.x; e < tot; e += HL_BLOCK) {
      double v = it.A ? it.scale * it.A[e] : 0.0;
      if (it.add_identity && (e % it.m) == (e / it.m)) v += 1.0;
      it.dA[e] = v;
    }
    return;
  }
  const int k = (it.A && it.rank) ? *it.rank : 0;
  for (int e = threadIdx.x; e < it.m * k; e += HL_BLOCK) it.dA[e] = it.scale * it.A[e];
  for (int e = threadIdx.x; e < it.n * k; e += HL_BLOCK) it.dB[e] = it.B[e];
  if (threadIdx.x == 0 && it.drank) *it.drank = k;
}

// LU without pivoting of a diagonal leaf (in place), then the inverses of the
// unit-lower factor and of the upper factor.
__global__ void __launch_bounds__(HL_BLOCK) k_getrf_inv(const GetrfItem* items, int32_t* zero_pivot) {
  __shared__ double A[64 * 64];
  __shared__ double X[64 * 64];
  const GetrfItem it = items[blockIdx.x];
  const int m = it.m;
  for (int e = threadIdx.x; e < m * m; e += HL_BLOCK) A[e] = it.LU[e];
  __syncthreads();
  for (int kk = 0; kk < m; ++kk) {
    const double piv = A[kk + m * kk];
    if (piv == 0.0) {
      if (threadIdx.x == 0) atomicAdd(zero_pivot, 1);
      return;
    }
    for (int i = kk + 1 + threadIdx.x; i < m; i += HL_BLOCK) A[i + m * kk] /= piv;
    __syncthreads();
    const int rem = m - kk - 1;
    for (int e = threadIdx.x; e < rem * rem; e += HL_BLOCK) {
      int i = kk + 1 + e % rem, j = kk + 1 + e / rem;
      A[i + m * j] -= A[i + m * kk] * A[kk + m * j];
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < m * m; e += HL_BLOCK) it.LU[e] = A[e];
  // inverse of the unit lower factor: column c by forward substitution
  for (int c = threadIdx.x; c < m; c += HL_BLOCK) {
    for (int i = 0; i < m; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      if (i > c)
        for (int j = c; j < i; ++j) v -= A[i + m * j] * X[j + m * c];
      X[i + m * c] = (i < c) ? 0.0 : v;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m * m; e += HL_BLOCK) it.Li[e] = X[e];
  __syncthreads();
  // inverse of the upper factor: column c by backward substitution
  for (int c = threadIdx.x; c < m; c += HL_BLOCK) {
    for (int i = m - 1; i >= 0; --i) {
      double v = 0.0;
      if (i <= c) {
        v = (i == c) ? 1.0 : 0.0;
        for (int j = i + 1; j <= c; ++j) v -= A[i + m * j] * X[j + m * c];
        v /= A[i + m * i];
      }
      X[i + m * c] = v;
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < m * m; e += HL_BLOCK) it.Ui[e] = X[e];
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

__global__ void __launch_bounds__(HL_BLOCK) k_apply_gather(const ApplyJob* jobs, const GatherItem* items,
                                                           DevLists dl) {
  __shared__ double Xs[64 * KMAX];
  const GatherItem it = items[blockIdx.x];
  const ApplyJob J = jobs[it.job];
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
        if (!J.trans) {
          const double* D = d.A + (lo - d.rlo);
          for (int u = 0; qg + 4 * u < kx; ++u) {
            int q = qg + 4 * u;
            double s = 0.0;
            for (int j = 0; j < len; ++j) s += D[i + (size_t)d.m * j] * Xs[j + len * q];
            acc[u] += s;
          }
        } else {
          const double* D = d.A + (size_t)d.m * (lo - d.clo);
          for (int u = 0; qg + 4 * u < kx; ++u) {
            int q = qg + 4 * u;
            double s = 0.0;
            for (int j = 0; j < len; ++j) s += D[j + (size_t)d.m * i] * Xs[j + len * q];
            acc[u] += s;
          }
        }
      }
    } else {
      const int k = J.rank[l];
      const double* Tl = J.T + (size_t)(l - J.lbeg) * J.tstride;
      if (i < mr) {
        const double* F = J.trans ? d.B + (lo - d.clo) : d.A + (lo - d.rlo);
        const int ld = J.trans ? d.n : d.m;
        for (int u = 0; qg + 4 * u < kx; ++u) {
          int q = qg + 4 * u;
          double s = 0.0;
          for (int p = 0; p < k; ++p) s += F[i + (size_t)ld * p] * Tl[p + d.kcap * q];
          acc[u] += s;
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
hipError_t launch_aca(const ProblemDev& P, const int32_t* perm, const LeafDesc* L, const int32_t* ids,
                      int n, double* U, double* V, const int64_t* uoff, const int64_t* voff,
                      int32_t* ranks, int kcap, double eps, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_aca, dim3(n), dim3(HL_BLOCK), 0, s, P, perm, L, ids, U, V, uoff, voff, ranks,
                     kcap, eps);
  return post();
}
hipError_t launch_flush_lr(const LFlushTarget* tg, int ntg, const Term* terms, const ChunkItem* gram,
                           int ngram, const ChunkItem* expand, int nexp, double tol, hipStream_t s) {
  if (ntg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_flush_gram, dim3(ngram), dim3(HL_BLOCK), 0, s, tg, terms, gram);
  size_t shm = 4 * KMAX * KMAX * sizeof(double);
  hipLaunchKernelGGL(k_flush_core, dim3(ntg), dim3(HL_BLOCK), shm, s, tg, terms, tol);
  hipLaunchKernelGGL(k_flush_expand, dim3(nexp), dim3(HL_BLOCK), 0, s, tg, terms, expand);
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
hipError_t launch_getrf_inv(const GetrfItem* items, int n, int32_t* zero_pivot, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_getrf_inv, dim3(n), dim3(HL_BLOCK), 0, s, items, zero_pivot);
  return post();
}
hipError_t launch_apply(const ApplyJob* jobs, const ProjItem* proj, int nproj, const GatherItem* gat,
                        int ngat, const DevLists& dl, hipStream_t s) {
  if (nproj > 0) hipLaunchKernelGGL(k_apply_proj, dim3(nproj), dim3(HL_BLOCK), 0, s, jobs, proj);
  if (ngat > 0) hipLaunchKernelGGL(k_apply_gather, dim3(ngat), dim3(HL_BLOCK), 0, s, jobs, gat, dl);
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
hipError_t launch_densify(const LeafDesc* L, const int32_t* rank, int nleaves, const int32_t* perm,
                          int N, double* dense, hipStream_t s) {
  hipLaunchKernelGGL(k_densify, dim3(nleaves), dim3(HL_BLOCK), 0, s, L, rank, perm, N, dense);
  return post();
}

}  // namespace hl

namespace hl {
hipError_t init_kernel_attributes() {
  return hipFuncSetAttribute((const void*)k_flush_core, hipFuncAttributeMaxDynamicSharedMemorySize,
                             4 * KMAX * KMAX * (int)sizeof(double));
}
}  // namespace hl
