// Per-step H-matrix-vector product (App. B.2: dense leaves by GEMV, low-rank
// leaves as U (V^T x)), the HBM-bound hot loop of every Crank-Nicolson step.
//
// Two launches, no atomics, fixed summation order:
//  1. k_mv_project: one wavefront per segment (<= MV_SEG rows of one V),
//     partial[seg][p] = sum_j V[j, p] x[j].
//  2. k_mv_gather: one workgroup per leaf cluster rho (owner computes);
//     y_rho = sum_dense D x + sum_lowrank U[rho, :] t, t = sum of the leaf's
//     segment partials; four wavefronts split the columns, then reduce in
//     LDS and apply the Crank-Nicolson epilogue.
#include <hip/hip_runtime.h>

#include "hl_mv.h"

namespace hl {

__device__ __forceinline__ double mv_warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <typename TL>
__global__ void __launch_bounds__(256) k_mv_project(const MvSeg* segs, int nseg, const double* x,
                                                    double* partial) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int sidx = blockIdx.x * 4 + w;
  if (sidx >= nseg) return;
  const MvSeg S = segs[sidx];
  const TL* V = reinterpret_cast<const TL*>(S.V);
  double acc[MV_KP];
#pragma unroll
  for (int p = 0; p < MV_KP; ++p) acc[p] = 0.0;
  for (int j = S.r0 + lane; j < S.r1; j += 64) {
    const double xv = x[S.xoff + j];
#pragma unroll
    for (int p = 0; p < MV_KP; ++p)
      if (p < S.k) acc[p] += (double)V[j + (size_t)S.ld * p] * xv;
  }
#pragma unroll
  for (int p = 0; p < MV_KP; ++p) {
    if (p < S.k) {
      double s = mv_warp_sum(acc[p]);
      if (lane == 0) partial[(size_t)sidx * MV_KP + p] = s;
    }
  }
}

template <typename TD, typename TL>
__global__ void __launch_bounds__(256) k_mv_gather(const MvRow* rows, const MvEntry* ents, const double* x,
                                                   const double* partial, MvEpi epi) {
  __shared__ double red[4][64];
  const MvRow R = rows[blockIdx.x];
  const int i = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int mr = R.hi - R.lo;
  const int ii = i < mr ? i : mr - 1;   // clamped row: loads stay in bounds, result discarded
  double acc = 0.0;
  for (int e = R.ebeg; e < R.eend; ++e) {
    const MvEntry E = ents[e];
    if (E.kind == 0) {
      // wavefront g owns columns [16 g, 16 g + 16): 16 independent loads in flight
      const TD* D = reinterpret_cast<const TD*>(E.ptr) + ii;
      const double* xs = x + E.xoff;
      const int j0 = 16 * g;
      if (j0 + 16 <= E.n) {
        double dv[16], xv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
          dv[q] = (double)D[(size_t)E.ld * (j0 + q)];
          xv[q] = xs[j0 + q];
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) acc += dv[q] * xv[q];
      } else {
        for (int j = j0; j < E.n && j < j0 + 16; ++j) acc += (double)D[(size_t)E.ld * j] * xs[j];
        for (int j = 64 + g; j < E.n; j += 4) acc += (double)D[(size_t)E.ld * j] * xs[j];
      }
    } else {
      const TL* U = reinterpret_cast<const TL*>(E.ptr) + ii;
      double uv[8], tv[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int p = g + 4 * q;
        uv[q] = 0.0;
        tv[q] = 0.0;
        if (p < E.k) {
          uv[q] = (double)U[(size_t)E.ld * p];
          double t = 0.0;
          for (int s = 0; s < E.nseg; ++s) t += partial[(size_t)(E.sbeg + s) * MV_KP + p];
          tv[q] = t;
        }
      }
#pragma unroll
      for (int q = 0; q < 8; ++q) acc += uv[q] * tv[q];
    }
  }
  red[g][i] = acc;
  __syncthreads();
  if (g == 0 && i < mr) {
    const double v = (red[0][i] + red[1][i]) + (red[2][i] + red[3][i]);
    const int r = R.lo + i;
    double out;
    switch (epi.kind) {
      case MV_EPI_RHS:   // b = u + hdt * G u + cg * g
        out = epi.u[r] + epi.hdt * v + (epi.g ? epi.cg * epi.g[r] : 0.0);
        break;
      case MV_EPI_RESID:  // r = b - (x - hdt * G x)
        out = epi.b[r] - (epi.u[r] - epi.hdt * v);
        break;
      case MV_EPI_ADD:    // y = u + A x (refinement update)
        out = epi.u[r] + v;
        break;
      default:
        out = v;
    }
    epi.y[r] = out;
  }
}

template <typename TD, typename TL>
hipError_t mv_launch_t(const MvDev& M, const double* x, double* partial, const MvEpi& epi, hipStream_t s) {
  if (M.nseg > 0)
    hipLaunchKernelGGL(k_mv_project<TL>, dim3((M.nseg + 3) / 4), dim3(256), 0, s, M.segs, M.nseg, x, partial);
  hipLaunchKernelGGL((k_mv_gather<TD, TL>), dim3(M.nrows), dim3(256), 0, s, M.rows, M.ents, x, partial, epi);
  return hipGetLastError();
}

hipError_t mv_launch(const MvDev& M, const double* x, double* partial, const MvEpi& epi, hipStream_t s) {
  if (M.dense_f32) {
    if (M.lr_f32) return mv_launch_t<float, float>(M, x, partial, epi, s);
    return mv_launch_t<float, double>(M, x, partial, epi, s);
  }
  if (M.lr_f32) return mv_launch_t<double, float>(M, x, partial, epi, s);
  return mv_launch_t<double, double>(M, x, partial, epi, s);
}

hipError_t project_launch(const MvDev& M, const double* x, double* partial, hipStream_t s) {
  if (M.nseg == 0) return hipSuccess;
  if (M.lr_f32)
    hipLaunchKernelGGL(k_mv_project<float>, dim3((M.nseg + 3) / 4), dim3(256), 0, s, M.segs, M.nseg, x, partial);
  else
    hipLaunchKernelGGL(k_mv_project<double>, dim3((M.nseg + 3) / 4), dim3(256), 0, s, M.segs, M.nseg, x, partial);
  return hipGetLastError();
}

hipError_t gather_launch(const MvDev& M, const double* x, const double* partial, const MvEpi& epi, hipStream_t s) {
  if (M.dense_f32 && M.lr_f32)
    hipLaunchKernelGGL((k_mv_gather<float, float>), dim3(M.nrows), dim3(256), 0, s, M.rows, M.ents, x, partial, epi);
  else if (M.dense_f32)
    hipLaunchKernelGGL((k_mv_gather<float, double>), dim3(M.nrows), dim3(256), 0, s, M.rows, M.ents, x, partial, epi);
  else if (M.lr_f32)
    hipLaunchKernelGGL((k_mv_gather<double, float>), dim3(M.nrows), dim3(256), 0, s, M.rows, M.ents, x, partial, epi);
  else
    hipLaunchKernelGGL((k_mv_gather<double, double>), dim3(M.nrows), dim3(256), 0, s, M.rows, M.ents, x, partial, epi);
  return hipGetLastError();
}

__global__ void k_convert_f32(const double* in, float* out, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) out[i] = (float)in[i];
}

hipError_t launch_convert_f32(const double* in, float* out, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_convert_f32, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

}  // namespace hl
