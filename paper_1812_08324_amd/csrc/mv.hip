// Per-step H-matrix-vector product (App. B.2: dense leaves by GEMV, low-rank
// leaves as U (V^T x)), the HBM-bound hot loop of every Crank-Nicolson step.
//
// Two launches, no atomics, fixed summation order:
//  1. k_mv_project (blocks of 16 wavefronts): t_b = V_b^T x for every
//     low-rank leaf b.  A small leaf (<= MV_SMALL rows) is one wavefront;
//     a large one is split over the 16 wavefronts of a block and reduced in
//     LDS.  Lanes run along the rows (coalesced); a lane issues the loads of
//     8 columns and two rows before accumulating.
//  2. k_mv_gather: one workgroup per leaf cluster rho (owner computes):
//     y_rho = sum_dense D x + sum_lowrank U[rho, :] t_b; the row's entry list
//     is staged in LDS, the four wavefronts take entries round-robin, then
//     reduce in LDS and apply the Crank-Nicolson epilogue.
#include <hip/hip_runtime.h>

#include "hl_mv.h"

namespace hl {

__device__ __forceinline__ double mv_warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum_{j in [r0, r1)} V[j, cg + q] x[j] for q < 8, this lane's share (rows lane + 64 i)
template <typename TL>
__device__ __forceinline__ void proj_part(const TL* V, int ld, const double* xs, int r0, int r1, int k, int cg,
                                          int lane, double acc[8]) {
#pragma unroll
  for (int q = 0; q < 8; ++q) acc[q] = 0.0;
  int j = r0 + lane;
  for (; j + 64 < r1; j += 128) {
    const double x0 = xs[j], x1 = xs[j + 64];
    double v0[8], v1[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      v0[q] = cg + q < k ? (double)V[j + (size_t)ld * (cg + q)] : 0.0;
      v1[q] = cg + q < k ? (double)V[j + 64 + (size_t)ld * (cg + q)] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) acc[q] += v0[q] * x0 + v1[q] * x1;
  }
  if (j < r1) {
    const double x0 = xs[j];
#pragma unroll
    for (int q = 0; q < 8; ++q)
      if (cg + q < k) acc[q] += (double)V[j + (size_t)ld * (cg + q)] * x0;
  }
}

template <typename TL>
__global__ void __launch_bounds__(1024) k_mv_project(const MvSeg* segs, const MvProjBlock* pblk, const double* x,
                                                     double* tb) {
  __shared__ double red[16][MV_KP];
  const MvProjBlock B = pblk[blockIdx.x];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (!B.big) {
    if (w >= B.count) return;
    const MvSeg S = segs[B.first + w];
    const TL* V = reinterpret_cast<const TL*>(S.V);
    for (int cg = 0; cg < S.k; cg += 8) {
      double acc[8];
      proj_part<TL>(V, S.ld, x + S.xoff, 0, S.n, S.k, cg, lane, acc);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        if (cg + q < S.k) {
          const double s = mv_warp_sum(acc[q]);
          if (lane == 0) tb[(size_t)S.tb * MV_KP + cg + q] = s;
        }
      }
    }
    return;
  }
  const MvSeg S = segs[B.first];
  const TL* V = reinterpret_cast<const TL*>(S.V);
  const int chunk = (((S.n + 15) / 16) + 63) & ~63;   // rows per wavefront, multiple of 64
  const int r0 = min(S.n, w * chunk), r1 = min(S.n, r0 + chunk);
  for (int cg = 0; cg < S.k; cg += 8) {
    double acc[8];
    proj_part<TL>(V, S.ld, x + S.xoff, r0, r1, S.k, cg, lane, acc);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double s = mv_warp_sum(acc[q]);
      if (lane == 0 && cg + q < MV_KP) red[w][cg + q] = s;
    }
  }
  __syncthreads();
  if (threadIdx.x < S.k) {
    double s = 0.0;
    for (int g = 0; g < 16; ++g) s += red[g][threadIdx.x];
    tb[(size_t)S.tb * MV_KP + threadIdx.x] = s;
  }
}

template <typename TD, typename TL>
__global__ void __launch_bounds__(256) k_mv_gather(const MvRow* rows, const MvEntry* ents, const double* x,
                                                   const double* tb, MvEpi epi) {
  constexpr int EMAX = 128;
  __shared__ double red[4][64];
  __shared__ MvEntry se[EMAX];
  const MvRow R = rows[blockIdx.x];
  const int i = threadIdx.x & 63, g = threadIdx.x >> 6;
  const int mr = R.hi - R.lo;
  const int ii = i < mr ? i : mr - 1;   // clamped row: loads stay in bounds, result discarded
  double acc = 0.0;
  for (int base = R.ebeg; base < R.eend; base += EMAX) {
    const int cnt = min(EMAX, R.eend - base);
    __syncthreads();
    {
      // stage the entry list (8-byte words) in LDS
      const long long* src = reinterpret_cast<const long long*>(ents + base);
      long long* dst = reinterpret_cast<long long*>(se);
      const int words = cnt * (int)(sizeof(MvEntry) / 8);
      for (int e = threadIdx.x; e < words; e += 256) dst[e] = src[e];
    }
    __syncthreads();
    for (int e = g; e < cnt; e += 4) {
      const MvEntry E = se[e];
      if (E.kind == 0) {
        const TD* D = reinterpret_cast<const TD*>(E.ptr) + ii;
        const double* xs = x + E.xoff;
        int j = 0;
        for (; j + 16 <= E.n; j += 16) {
          double dv[16], xv[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) {
            dv[q] = (double)D[(size_t)E.ld * (j + q)];
            xv[q] = xs[j + q];
          }
#pragma unroll
          for (int q = 0; q < 16; ++q) acc += dv[q] * xv[q];
        }
        for (; j < E.n; ++j) acc += (double)D[(size_t)E.ld * j] * xs[j];
      } else {
        const TL* U = reinterpret_cast<const TL*>(E.ptr) + ii;
        const double* t = tb + (size_t)E.tb * MV_KP;
        for (int p = 0; p < E.k; p += 8) {
          double uv[8], tv[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            uv[q] = p + q < E.k ? (double)U[(size_t)E.ld * (p + q)] : 0.0;
            tv[q] = p + q < E.k ? t[p + q] : 0.0;
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) acc += uv[q] * tv[q];
        }
      }
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
hipError_t mv_launch_t(const MvDev& M, const double* x, double* tb, const MvEpi& epi, hipStream_t s) {
  if (M.npblk > 0)
    hipLaunchKernelGGL(k_mv_project<TL>, dim3(M.npblk), dim3(1024), 0, s, M.segs, M.pblk, x, M.tb);
  hipLaunchKernelGGL((k_mv_gather<TD, TL>), dim3(M.nrows), dim3(256), 0, s, M.rows, M.ents, x, M.tb, epi);
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

hipError_t project_launch(const MvDev& M, const double* x, double* tb, hipStream_t s) {
  (void)tb;
  if (M.npblk == 0) return hipSuccess;
  if (M.lr_f32)
    hipLaunchKernelGGL(k_mv_project<float>, dim3(M.npblk), dim3(1024), 0, s, M.segs, M.pblk, x, M.tb);
  else
    hipLaunchKernelGGL(k_mv_project<double>, dim3(M.npblk), dim3(1024), 0, s, M.segs, M.pblk, x, M.tb);
  return hipGetLastError();
}

hipError_t gather_launch(const MvDev& M, const double* x, const double* partial, const MvEpi& epi, hipStream_t s) {
  if (M.dense_f32 && M.lr_f32)
    hipLaunchKernelGGL((k_mv_gather<float, float>), dim3(M.nrows), dim3(256), 0, s, M.rows, M.ents, x, M.tb, epi);
  else if (M.dense_f32)
    hipLaunchKernelGGL((k_mv_gather<float, double>), dim3(M.nrows), dim3(256), 0, s, M.rows, M.ents, x, M.tb, epi);
  else if (M.lr_f32)
    hipLaunchKernelGGL((k_mv_gather<double, float>), dim3(M.nrows), dim3(256), 0, s, M.rows, M.ents, x, M.tb, epi);
  else
    hipLaunchKernelGGL((k_mv_gather<double, double>), dim3(M.nrows), dim3(256), 0, s, M.rows, M.ents, x, M.tb, epi);
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
