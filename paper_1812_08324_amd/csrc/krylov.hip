// Vector kernels of the Krylov iterations (conjugate gradients and
// BiCGSTAB) that the factorised H-matrix preconditions (Sec. 5.1; Sec. 5.3
// solves the fractional Poisson problem by conjugate gradients).  The
// iteration's scalars stay on the device: dot products are reduced into a
// scalar array in a fixed order (deterministic), derived coefficients are
// formed there by one thread, and the vector updates read them, so an
// iteration needs one host read-back (the residual norm) and no other
// synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "hl_kernels.h"

namespace hl {

namespace {

constexpr int KB = 256;   // threads per block (four wavefronts)

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum over the 256-thread block in a fixed order; valid in thread 0
__device__ __forceinline__ double block_total(double v, double* red) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double s = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return s;
}

__device__ __forceinline__ double coef(const KrCoef& c, const double* sc) {
  return c.idx >= 0 ? c.mul * sc[c.idx] : c.mul;
}

// partial[k * gridDim.x + block] = sum over the block's rows of a_k b_k
__global__ void __launch_bounds__(KB) k_kr_dot_partial(KrDots d, int N, double* partial) {
  __shared__ double red[4];
  double acc[KR_MAXDOT];
#pragma unroll
  for (int k = 0; k < KR_MAXDOT; ++k) acc[k] = 0.0;
  for (int i = blockIdx.x * KB + threadIdx.x; i < N; i += gridDim.x * KB) {
#pragma unroll
    for (int k = 0; k < KR_MAXDOT; ++k)
      if (k < d.n) acc[k] += d.a[k][i] * d.b[k][i];
  }
#pragma unroll
  for (int k = 0; k < KR_MAXDOT; ++k) {
    if (k >= d.n) break;
    const double t = block_total(acc[k], red);
    if (threadIdx.x == 0) partial[k * gridDim.x + blockIdx.x] = t;
  }
}

// sc[d.out[k]] = sum of the nb partials of dot k, in block order
__global__ void __launch_bounds__(KB) k_kr_dot_final(KrDots d, const double* partial, int nb, double* sc) {
  __shared__ double red[4];
  for (int k = 0; k < d.n; ++k) {
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += KB) a += partial[k * nb + i];
    const double t = block_total(a, red);
    if (threadIdx.x == 0) sc[d.out[k]] = t;
  }
}

// in order: sc[dst] = (sc[num] / sc[den]) * (sc[num2] / sc[den2]), then
// sc[copy_to] = sc[copy_from] (a value kept for the next iteration)
__global__ void k_kr_scalars(KrRatios q, double* sc) {
  for (int k = 0; k < q.n; ++k) {
    const KrRatio r = q.r[k];
    double v = sc[r.num] / sc[r.den];
    if (r.num2 >= 0) v *= sc[r.num2] / sc[r.den2];
    sc[r.dst] = v;
    if (r.copy_from >= 0) sc[r.copy_to] = sc[r.copy_from];
  }
}

// out = c0 x0 + c1 x1 + c2 x2 (x_k may be null; out may alias any x_k:
// every row is read and written by one thread)
__global__ void __launch_bounds__(KB) k_kr_comb(double* out, const double* x0, KrCoef c0, const double* x1,
                                                KrCoef c1, const double* x2, KrCoef c2, const double* sc, int N) {
  const int i = blockIdx.x * KB + threadIdx.x;
  if (i >= N) return;
  double v = coef(c0, sc) * x0[i];
  if (x1) v += coef(c1, sc) * x1[i];
  if (x2) v += coef(c2, sc) * x2[i];
  out[i] = v;
}

// GMRES (classical Gram-Schmidt, applied twice): partial[c * gridDim.x +
// block] = sum over the block's rows of V[c ld + i] w[i], c < ncol
__global__ void __launch_bounds__(KB) k_gm_dot_partial(const double* V, int ld, int ncol, const double* w, int N,
                                                       double* partial) {
  __shared__ double red[4];
  for (int c = 0; c < ncol; ++c) {
    const double* vc = V + (size_t)c * ld;
    double acc = 0.0;
    for (int i = blockIdx.x * KB + threadIdx.x; i < N; i += gridDim.x * KB) acc += vc[i] * w[i];
    const double tsum = block_total(acc, red);
    if (threadIdx.x == 0) partial[(size_t)c * gridDim.x + blockIdx.x] = tsum;
  }
}

// out[c] = sum of the nb partials of column c, in block order
__global__ void __launch_bounds__(KB) k_gm_dot_final(const double* partial, int nb, int ncol, double* out) {
  __shared__ double red[4];
  for (int c = 0; c < ncol; ++c) {
    double a = 0.0;
    for (int i = threadIdx.x; i < nb; i += KB) a += partial[(size_t)c * nb + i];
    const double tsum = block_total(a, red);
    if (threadIdx.x == 0) out[c] = tsum;
  }
}

// out[i] = (base ? base[i] : 0) + sign * sum_{c < ncol} coef[c] V[c ld + i]
// (c in increasing order; out may alias base)
__global__ void __launch_bounds__(KB) k_gm_comb(double* out, const double* base, const double* V, int ld, int ncol,
                                                const double* coef, double sign, int N) {
  const int i = blockIdx.x * KB + threadIdx.x;
  if (i >= N) return;
  double acc = 0.0;
  for (int c = 0; c < ncol; ++c) acc += coef[c] * V[(size_t)c * ld + i];
  out[i] = (base ? base[i] : 0.0) + sign * acc;
}

}  // namespace

hipError_t launch_gm_dots(const double* V, int ld, int ncol, const double* w, int N, double* partial, double* out,
                          hipStream_t s) {
  if (ncol < 1) return hipErrorInvalidValue;
  const int nb = kr_blocks(N);
  hipLaunchKernelGGL(k_gm_dot_partial, dim3(nb), dim3(KB), 0, s, V, ld, ncol, w, N, partial);
  hipLaunchKernelGGL(k_gm_dot_final, dim3(1), dim3(KB), 0, s, partial, nb, ncol, out);
  return hipGetLastError();
}

hipError_t launch_gm_comb(double* out, const double* base, const double* V, int ld, int ncol, const double* coef,
                          double sign, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_gm_comb, dim3((N + KB - 1) / KB), dim3(KB), 0, s, out, base, V, ld, ncol, coef, sign, N);
  return hipGetLastError();
}

int kr_blocks(int N) { return std::min(512, std::max(1, (N + KB - 1) / KB)); }

hipError_t launch_kr_dots(const KrDots& d, int N, double* partial, double* sc, hipStream_t s) {
  if (d.n < 1 || d.n > KR_MAXDOT) return hipErrorInvalidValue;
  const int nb = kr_blocks(N);
  hipLaunchKernelGGL(k_kr_dot_partial, dim3(nb), dim3(KB), 0, s, d, N, partial);
  hipLaunchKernelGGL(k_kr_dot_final, dim3(1), dim3(KB), 0, s, d, partial, nb, sc);
  return hipGetLastError();
}

hipError_t launch_kr_scalars(const KrRatios& q, double* sc, hipStream_t s) {
  if (q.n < 1 || q.n > KR_MAXRATIO) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_kr_scalars, dim3(1), dim3(1), 0, s, q, sc);
  return hipGetLastError();
}

hipError_t launch_kr_comb(double* out, const double* x0, KrCoef c0, const double* x1, KrCoef c1,
                          const double* x2, KrCoef c2, const double* sc, int N, hipStream_t s) {
  hipLaunchKernelGGL(k_kr_comb, dim3((N + KB - 1) / KB), dim3(KB), 0, s, out, x0, c0, x1, c1, x2, c2, sc, N);
  return hipGetLastError();
}

}  // namespace hl
