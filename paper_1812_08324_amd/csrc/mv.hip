// Per-step H-matrix-vector product (App. B.2: dense leaves by GEMV, low-rank
// leaves as U (V^T x)), the HBM-bound hot loop of every Crank-Nicolson step.
//
// Two launches, no atomics, fixed summation order:
//  1. k_mv_project: every wavefront owns one tile (a row range of one V
//     factor; a leaf has at most MV_PMAX tiles).  Lanes run along the rows
//     (coalesced), each lane issues the loads of RPL rows x all k columns
//     before accumulating, and a transposed butterfly reduces the k column
//     sums across the 64 lanes with k + log steps instead of 6 k.  The k
//     partial sums of the tile go to its slot of the partial buffer.
//  2. k_mv_gather: one workgroup per leaf cluster rho (owner computes):
//     y_rho = sum_dense D x + sum_lowrank U[rho, :] t_b.  The wavefronts take
//     entries round-robin (the host sorts each list by bytes and splits dense
//     leaves into 16-column pieces); a wavefront forms t_b = sum of the
//     leaf's partials in a fixed order itself, with its U loads in flight.
//     The wavefronts reduce in LDS and apply the Crank-Nicolson epilogue.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "hl_mv.h"

namespace hl {

// ---------------------------------------------------------------------------
// transposed butterfly: a[0..W) per lane -> lane holds, in a[0], the sum over
// all 64 lanes of column (lane / (64 / W)) of the original arrays.
// ---------------------------------------------------------------------------
template <int W, int O>
struct ColReduce {
  static __device__ __forceinline__ void run(double* a, int lane) {
    constexpr int H = W / 2;
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const double send = up ? a[i] : a[i + H];
      const double keep = up ? a[i + H] : a[i];
      a[i] = keep + __shfl_xor(send, O, 64);
    }
    ColReduce<H, O / 2>::run(a, lane);
  }
};
template <int O>
struct ColReduce<1, O> {
  static __device__ __forceinline__ void run(double* a, int lane) {
    a[0] += __shfl_xor(a[0], O, 64);
    ColReduce<1, O / 2>::run(a, lane);
  }
};
template <>
struct ColReduce<1, 0> {
  static __device__ __forceinline__ void run(double*, int) {}
};

// value of `v` in lane l (l uniform across the wavefront)
__device__ __forceinline__ double bcast_lane(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// wavefront-uniform copies (scalar registers) of values the compiler cannot
// prove uniform
__device__ __forceinline__ int wuni(int v) { return __builtin_amdgcn_readfirstlane(v); }
// Leaf data lives in device global memory: addressing it through the global
// address space lets the loads take a scalar base plus a 32-bit lane offset.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> wuni_ptr(const void* p) {
  const unsigned long long b = (unsigned long long)p;
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)b);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(b >> 32));
  return (gptr<T>)(((unsigned long long)hi << 32) | lo);
}

// A BF16 value is stored as the high 16 bits of an FP32 and widened exactly
// on use; the products accumulate in FP64 like the other precisions.
using bf16 = uint16_t;
__device__ __forceinline__ double to_d(double v) { return v; }
__device__ __forceinline__ double to_d(float v) { return (double)v; }
__device__ __forceinline__ double to_d(bf16 v) { return (double)__uint_as_float((uint32_t)v << 16); }

template <typename TL, int KB>
constexpr int rows_per_lane() {
  // 64 VGPRs of loads in flight per lane (a BF16 value takes one register too)
  return (sizeof(TL) <= 4 ? 64 : 32) / KB;
}

// one projection tile (V in precision TL): the k partial sums of the
// wavefront's rows, written to the tile's slot
template <typename TL, int KB, int SB = KB, int RPL = rows_per_lane<TL, KB>()>
__device__ __forceinline__ void project_tile(const MvTile& T, const double* __restrict__ x, double* __restrict__ part,
                                             int lane) {
  const gptr<TL> V = wuni_ptr<TL>(T.V);
  const double* __restrict__ xs = x + T.xoff;
  double acc[KB];
#pragma unroll
  for (int q = 0; q < KB; ++q) acc[q] = 0.0;
  for (int r = 0; r < T.n; r += 64 * RPL) {
    TL v[RPL][KB];
    double xv[RPL];
    // Every load is unconditional, so all of them are in flight before the
    // first use: rows past the tile read row 0 (x weight 0) and columns past
    // the rank re-read column k-1 (their sums land in columns >= k, which
    // are never stored).
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int j = r + u * 64 + lane;
      const bool ok = j < T.n;
      const int jj = ok ? j : 0;
      const double xr = xs[jj];
      xv[u] = ok ? xr : 0.0;
#pragma unroll
      for (int q = 0; q < KB; ++q) v[u][q] = V[(unsigned)(jj + T.ld * min(q, T.k - 1))];
    }
#pragma unroll
    for (int u = 0; u < RPL; ++u)
#pragma unroll
      for (int q = 0; q < KB; ++q) acc[q] += to_d(v[u][q]) * xv[u];
  }
  ColReduce<KB, 32>::run(acc, lane);
  constexpr int G = 64 / KB;
  const int col = lane / G;
  if (lane % G == 0 && col < T.k) part[(size_t)T.slot * SB + T.col0 + col] = acc[0];
}

template <int KB, int SB = KB>
__device__ __forceinline__ void project_any(const MvTile& T, const double* __restrict__ x,
                                            double* __restrict__ part, int lane) {
  // tiles of at most 64 rows (leaves of the finest level) take one row per
  // lane: the full pass would load RPL - 1 rows that are never used
  const int fmt = wuni(T.f32), short_tile = wuni(T.n) <= 64;
  if (fmt == MV_FMT_BF16)
    short_tile ? project_tile<bf16, KB, SB, 1>(T, x, part, lane) : project_tile<bf16, KB, SB>(T, x, part, lane);
  else if (fmt == MV_FMT_F32)
    short_tile ? project_tile<float, KB, SB, 1>(T, x, part, lane) : project_tile<float, KB, SB>(T, x, part, lane);
  else
    short_tile ? project_tile<double, KB, SB, 1>(T, x, part, lane) : project_tile<double, KB, SB>(T, x, part, lane);
}

// KB: columns per wavefront (registers); SB: partial slot stride (the
// plan's rank bucket)
template <int KB, int SB>
__global__ void __launch_bounds__(256) k_mv_project(const MvTile* __restrict__ tiles, int ntiles,
                                                    const double* __restrict__ x, double* __restrict__ part) {
  const int wid = wuni(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (wid >= ntiles) return;   // the whole wavefront leaves; no block barrier below
  const MvTile T = tiles[wid];
  project_any<KB, SB>(T, x, part, threadIdx.x & 63);
}

constexpr int MV_GW = 8;   // wavefronts per gather workgroup

// y[r] = epilogue of the product's row value v (see MvEpi)
__device__ __forceinline__ void epilogue(const MvEpi& epi, int r, double v) {
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
    case MV_EPI_AXPY:
      out = epi.hdt * v + (epi.g ? epi.cg * epi.g[r] : 0.0);
      break;
    case MV_EPI_CNRES:
      out = (2.0 * epi.u[r] + (epi.g ? epi.cg * epi.g[r] : 0.0)) - (epi.b[r] - epi.hdt * v);
      break;
    case MV_EPI_NEXT:
      out = (epi.b[r] + v) - epi.u[r];
      break;
    case MV_EPI_SUB:
      out = v - epi.u[r];
      break;
    default:
      out = v;
  }
  epi.y[r] = out;
}

// t_b entry of a low-rank leaf: the sum of its n <= MV_PMAX partials (stride
// apart) in slot order.  The loads of 16 slots are issued before their
// adds, so the sum costs one memory round trip per 16 partials instead of
// one per partial; the masked slots add zeros.
__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int n, int stride) {
  double s = 0.0;
  for (int c0 = 0; c0 < n; c0 += 16) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) v[u] = c0 + u < n ? p[(size_t)(c0 + u) * stride] : 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u) s += v[u];
  }
  return s;
}

template <int GW = MV_GW>
struct GatherLds {
  double red[GW][64];
};

// U rows of a low-rank entry times t_b, t_b formed by the wavefront itself
// while its U loads are in flight: lane (q, g) = q + KB g sums the partials
// g PPG .. g PPG + PPG - 1 of column q in slot order, a butterfly over the
// groups g gives every lane of column q the same total (the tree order is
// fixed), and the products are summed over q in order.
template <typename TL, int KB>
__device__ __forceinline__ double gather_lowrank_self(const MvEntry& E, int ii, int lane,
                                                      const double* __restrict__ part) {
  constexpr int NG = 64 / KB, PPG = MV_PMAX / NG;
  static_assert(MV_PMAX % NG == 0, "partials per group");
  const int ek = wuni(E.k), ld = wuni(E.ld), en = wuni(E.n);
  const gptr<TL> U = wuni_ptr<TL>(E.ptr);
  double uv[KB];
#pragma unroll
  for (int q = 0; q < KB; ++q) uv[q] = to_d(U[(unsigned)(ii + ld * min(q, ek - 1))]);
  const int q = lane % KB, c0 = (lane / KB) * PPG;
  const double* pp = part + (size_t)wuni(E.slot) * KB + q;
  double t = 0.0;   // zero past the rank: the products below multiply by it
  constexpr int PC = PPG < 8 ? PPG : 8;   // loads in flight per chunk (registers)
#pragma unroll
  for (int u0 = 0; u0 < PPG; u0 += PC) {
    double pv[PC];
#pragma unroll
    for (int u = 0; u < PC; ++u) {
      const int c = c0 + u0 + u;
      pv[u] = (q < ek && c < en) ? pp[(size_t)c * KB] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PC; ++u) t += pv[u];
  }
#pragma unroll
  for (int o = KB; o < 64; o <<= 1) t += __shfl_xor(t, o, 64);
  double acc = 0.0;
#pragma unroll
  for (int k = 0; k < KB; ++k) acc += uv[k] * bcast_lane(t, k);
  return acc;
}

// one leaf cluster: y[R] = epilogue(sum over the entries of R).  Wavefront
// g takes entries g, g + GW, ... straight from the entry list (wavefront-
// uniform loads, the next descriptor fetched while the current entry is
// processed); no barrier until the final reduction across wavefronts.
template <typename TD, int KB, int GW = MV_GW>
__device__ __forceinline__ void gather_rows(const MvRow& R, const MvEntry* __restrict__ ents,
                                            const double* __restrict__ x, const double* __restrict__ part,
                                            const MvEpi& epi, GatherLds<GW>& L) {
  const int i = threadIdx.x & 63, g = wuni(threadIdx.x >> 6);
  const int mr = R.hi - R.lo;
  const int ii = i < mr ? i : mr - 1;   // clamped row: loads stay in bounds, result discarded
  const int eend = wuni(R.eend);
  double acc = 0.0;
  int e = wuni(R.ebeg) + g;
  MvEntry En{};
  if (e < eend) En = ents[e];
  for (; e < eend; e += GW) {
    const MvEntry E = En;
    if (e + GW < eend) En = ents[e + GW];
    const int kind = wuni(E.kind), en = wuni(E.n), ld = wuni(E.ld);
    if (kind == 0) {
      const gptr<TD> D = wuni_ptr<TD>(E.ptr);
      const double xl = i < en ? x[wuni(E.xoff) + i] : 0.0;
      int j = 0;
      for (; j + 16 <= en; j += 16) {
        double dv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) dv[q] = to_d(D[(unsigned)(ii + ld * (j + q))]);
#pragma unroll
        for (int q = 0; q < 16; ++q) acc += dv[q] * bcast_lane(xl, j + q);
      }
      for (; j < en; ++j) acc += to_d(D[(unsigned)(ii + ld * j)]) * bcast_lane(xl, j);
    } else if (kind == 1) {
      acc += gather_lowrank_self<double, KB>(E, ii, i, part);
    } else if (kind == 2) {
      acc += gather_lowrank_self<float, KB>(E, ii, i, part);
    } else {
      acc += gather_lowrank_self<bf16, KB>(E, ii, i, part);
    }
  }
  L.red[g][i] = acc;
  __syncthreads();
  if (g == 0 && i < mr) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < GW; w += 2) v += L.red[w][i] + L.red[w + 1][i];
    epilogue(epi, R.lo + i, v);
  }
}

template <typename TD, int KB, int GW>
__global__ void __launch_bounds__(64 * GW) k_mv_gather(const MvRow* __restrict__ rows,
                                                       const MvEntry* __restrict__ ents,
                                                       const double* __restrict__ x,
                                                       const double* __restrict__ part, MvEpi epi) {
  __shared__ GatherLds<GW> L;
  const MvRow R = rows[blockIdx.x];
  gather_rows<TD, KB, GW>(R, ents, x, part, epi, L);
}

int project_rows_per_pass(int kb, bool narrow) {
  const int vals = narrow ? 64 : 32;
  return 64 * (vals / project_width(kb));
}

// Launches; with events, the events are attached to the dispatch itself
// (hipExtLaunchKernelGGL) and time exactly that kernel.
template <int KB>
static void project_t(const MvDev& M, const double* x, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (M.ntiles <= 0) return;
  // tiles of project_width(KB) columns into KB-wide partial slots
  constexpr int PK = project_width(KB);
  const dim3 grid((M.ntiles + 3) / 4);
  if (e0)
    hipExtLaunchKernelGGL((k_mv_project<PK, KB>), grid, dim3(256), 0, s, e0, e1, 0, M.tiles, M.ntiles, x, M.part);
  else
    hipLaunchKernelGGL((k_mv_project<PK, KB>), grid, dim3(256), 0, s, M.tiles, M.ntiles, x, M.part);
}

template <typename TD, int KB, int GW>
static void gather_w(const MvDev& M, const double* x, const MvEpi& epi, hipStream_t s, hipEvent_t e0,
                     hipEvent_t e1) {
  const dim3 grid(M.nrows), block(64 * GW);
  const double* part = M.part;
  if (e0)
    hipExtLaunchKernelGGL((k_mv_gather<TD, KB, GW>), grid, block, 0, s, e0, e1, 0, M.rows, M.ents, x, part, epi);
  else
    hipLaunchKernelGGL((k_mv_gather<TD, KB, GW>), grid, block, 0, s, M.rows, M.ents, x, part, epi);
}

template <typename TD, int KB>
static void gather_t(const MvDev& M, const double* x, const MvEpi& epi, hipStream_t s, hipEvent_t e0,
                     hipEvent_t e1) {
  if (M.nrows <= 0) return;
  if (M.gw == 4)
    gather_w<TD, KB, 4>(M, x, epi, s, e0, e1);
  else
    gather_w<TD, KB, MV_GW>(M, x, epi, s, e0, e1);
}

template <typename TD>
static void gather_kb(const MvDev& M, const double* x, const MvEpi& epi, hipStream_t s, hipEvent_t e0,
                      hipEvent_t e1) {
  if (M.kb <= 8)
    gather_t<TD, 8>(M, x, epi, s, e0, e1);
  else if (M.kb <= 16)
    gather_t<TD, 16>(M, x, epi, s, e0, e1);
  else
    gather_t<TD, 32>(M, x, epi, s, e0, e1);
}

hipError_t project_launch(const MvDev& M, const double* x, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  if (M.kb == 8)
    project_t<8>(M, x, s, e0, e1);
  else if (M.kb == 16)
    project_t<16>(M, x, s, e0, e1);
  else if (M.kb == 32)
    project_t<32>(M, x, s, e0, e1);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t gather_launch(const MvDev& M, const double* x, const MvEpi& epi, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1) {
  if (M.kb != 8 && M.kb != 16 && M.kb != 32) return hipErrorInvalidValue;
  if (M.gw != 4 && M.gw != MV_GW) return hipErrorInvalidValue;
  if (M.dense_f32)
    gather_kb<float>(M, x, epi, s, e0, e1);
  else
    gather_kb<double>(M, x, epi, s, e0, e1);
  return hipGetLastError();
}

hipError_t mv_launch(const MvDev& M, const double* x, const MvEpi& epi, hipStream_t s) {
  hipError_t e = project_launch(M, x, s);
  if (e != hipSuccess) return e;
  return gather_launch(M, x, epi, s);
}

// ---------------------------------------------------------------------------
// Batched products with up to R right-hand sides per problem (requests that
// share one operator): every matrix value is loaded once and applied to all
// member vectors.  A problem (MvInst) lists nr <= R members; member r takes
// part while its step limit exceeds the loop's step.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned member_mask(const MvInst& P, int step) {
  unsigned m = 0;
  const int nr = wuni(P.nr);
  for (int r = 0; r < nr; ++r)
    if (wuni(P.steps[r]) > step) m |= 1u << r;
  return m;
}

// projection tile for the members in `mask`: k partial sums per member
template <typename TL, int KB, int R, int SB>
__device__ __forceinline__ void project_tile_r(const MvTile& T, const MvInst& P, unsigned mask, int lane) {
  constexpr int RPL = rows_per_lane<TL, KB>();
  const gptr<TL> V = wuni_ptr<TL>(T.V);
  const double* xs[R];
#pragma unroll
  for (int r = 0; r < R; ++r) xs[r] = (mask >> r & 1u) ? P.x[r] + T.xoff : P.x[0] + T.xoff;
  double acc[R][KB];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < KB; ++q) acc[r][q] = 0.0;
  for (int r0 = 0; r0 < T.n; r0 += 64 * RPL) {
    TL v[RPL][KB];
    double xv[R][RPL];
    // unconditional loads (see project_tile); inactive members read member
    // 0's vector and are never stored
#pragma unroll
    for (int u = 0; u < RPL; ++u) {
      const int j = r0 + u * 64 + lane;
      const bool ok = j < T.n;
      const int jj = ok ? j : 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double xr = xs[r][jj];
        xv[r][u] = ok ? xr : 0.0;
      }
#pragma unroll
      for (int q = 0; q < KB; ++q) v[u][q] = V[(unsigned)(jj + T.ld * min(q, T.k - 1))];
    }
#pragma unroll
    for (int u = 0; u < RPL; ++u)
#pragma unroll
      for (int q = 0; q < KB; ++q) {
        const double vv = to_d(v[u][q]);
#pragma unroll
        for (int r = 0; r < R; ++r) acc[r][q] += vv * xv[r][u];
      }
  }
  constexpr int G = 64 / KB;
  const int col = lane / G;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (!(mask >> r & 1u)) continue;
    ColReduce<KB, 32>::run(acc[r], lane);
    if (lane % G == 0 && col < T.k) P.part[r][(size_t)T.slot * SB + T.col0 + col] = acc[r][0];
  }
}

template <int KB, int R, int SB>
__global__ void __launch_bounds__(256) k_mv_project_b(const MvInst* __restrict__ inst,
                                                      const MvRef* __restrict__ map, int nw, int step) {
  const int wid = wuni(blockIdx.x * 4 + (threadIdx.x >> 6));
  if (wid >= nw) return;   // whole wavefronts leave; no block barrier below
  const MvRef m = map[wid];
  const MvTile T = *reinterpret_cast<const MvTile*>(m.p);
  const MvInst& P = inst[wuni(m.inst)];
  const unsigned mask = member_mask(P, step);
  if (mask == 0) return;
  const int fmt = wuni(T.f32);
  if (fmt == MV_FMT_BF16)
    project_tile_r<bf16, KB, R, SB>(T, P, mask, threadIdx.x & 63);
  else if (fmt == MV_FMT_F32)
    project_tile_r<float, KB, R, SB>(T, P, mask, threadIdx.x & 63);
  else
    project_tile_r<double, KB, R, SB>(T, P, mask, threadIdx.x & 63);
}

// Batches mostly hold small problems with a few entries per leaf cluster,
// so the gather workgroups are by default half as wide as in the
// single-problem kernel (MV_GWB wavefronts) and twice as many stay resident
// per CU.
constexpr int MV_GWB = 4;

template <int KB, int R, int GWB>
struct GatherLdsR {
  static constexpr int E = MV_EMAX / R;   // entries staged per round
  double red[R][GWB][64];
  MvEntry se[E];
  double ts[R][E * KB];
};

template <typename TD, int KB, int R, int GWB>
__global__ void __launch_bounds__(64 * GWB) k_mv_gather_b(const MvInst* __restrict__ inst,
                                                          const MvRef* __restrict__ map, int step) {
  constexpr int MV_GWB = GWB;
  __shared__ GatherLdsR<KB, R, GWB> L;
  constexpr int E = GatherLdsR<KB, R, GWB>::E;
  const MvRef m = map[blockIdx.x];
  const MvRow Rw = *reinterpret_cast<const MvRow*>(m.p);
  const MvInst& P = inst[wuni(m.inst)];
  const unsigned mask = member_mask(P, step);
  if (mask == 0) return;   // whole workgroup, before any barrier
  const MvEntry* __restrict__ ents = P.dev.ents;
  const int i = threadIdx.x & 63, g = wuni(threadIdx.x >> 6);
  const int mr = Rw.hi - Rw.lo;
  const int ii = i < mr ? i : mr - 1;   // clamped row: loads stay in bounds, result discarded
  const double* xs[R];
#pragma unroll
  for (int r = 0; r < R; ++r) xs[r] = (mask >> r & 1u) ? P.x[r] : P.x[0];
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  for (int base = Rw.ebeg; base < Rw.eend; base += E) {
    const int cnt = min(E, Rw.eend - base);
    __syncthreads();
    {
      const long long* src = reinterpret_cast<const long long*>(ents + base);
      long long* dst = reinterpret_cast<long long*>(L.se);
      const int words = cnt * (int)(sizeof(MvEntry) / 8);
      for (int e = threadIdx.x; e < words; e += 64 * MV_GWB) dst[e] = src[e];
    }
    __syncthreads();
    // t_b of the low-rank entries per member: sum of its partials in slot order
    for (int it = threadIdx.x; it < R * cnt * KB; it += 64 * MV_GWB) {
      const int r = it / (cnt * KB), rem = it % (cnt * KB);
      const int e = rem / KB, q = rem % KB;
      const MvEntry& En = L.se[e];
      double s = 0.0;
      if ((mask >> r & 1u) && En.kind != 0 && q < En.k)
        s = sum_partials(P.part[r] + (size_t)En.slot * KB + q, En.n, KB);
      L.ts[r][rem] = s;
    }
    __syncthreads();
    for (int e = g; e < cnt; e += MV_GWB) {
      const int kind = wuni(L.se[e].kind), en = wuni(L.se[e].n), ek = wuni(L.se[e].k), ld = wuni(L.se[e].ld);
      if (kind == 0) {
        const gptr<TD> D = wuni_ptr<TD>(L.se[e].ptr);
        const int xo = wuni(L.se[e].xoff);
        double xl[R];
#pragma unroll
        for (int r = 0; r < R; ++r) xl[r] = i < en ? xs[r][xo + i] : 0.0;
        int j = 0;
        for (; j + 16 <= en; j += 16) {
          double dv[16];
#pragma unroll
          for (int q = 0; q < 16; ++q) dv[q] = to_d(D[(unsigned)(ii + ld * (j + q))]);
#pragma unroll
          for (int q = 0; q < 16; ++q)
#pragma unroll
            for (int r = 0; r < R; ++r) acc[r] += dv[q] * bcast_lane(xl[r], j + q);
        }
        for (; j < en; ++j) {
          const double dv = to_d(D[(unsigned)(ii + ld * j)]);
#pragma unroll
          for (int r = 0; r < R; ++r) acc[r] += dv * bcast_lane(xl[r], j);
        }
      } else {
        double uv[KB];
        if (kind == 1) {
          const gptr<double> U = wuni_ptr<double>(L.se[e].ptr);
#pragma unroll
          for (int q = 0; q < KB; ++q) uv[q] = U[(unsigned)(ii + ld * min(q, ek - 1))];
        } else if (kind == 2) {
          const gptr<float> U = wuni_ptr<float>(L.se[e].ptr);
#pragma unroll
          for (int q = 0; q < KB; ++q) uv[q] = to_d(U[(unsigned)(ii + ld * min(q, ek - 1))]);
        } else {
          const gptr<bf16> U = wuni_ptr<bf16>(L.se[e].ptr);
#pragma unroll
          for (int q = 0; q < KB; ++q) uv[q] = to_d(U[(unsigned)(ii + ld * min(q, ek - 1))]);
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          const double* t = L.ts[r] + e * KB;
          double a = 0.0;
#pragma unroll
          for (int q = 0; q < KB; ++q) a += uv[q] * t[q];
          acc[r] += a;
        }
      }
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) L.red[r][g][i] = acc[r];
  __syncthreads();
  if (g == 0 && i < mr) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (!(mask >> r & 1u)) continue;
      double v = 0.0;
#pragma unroll
      for (int w = 0; w < MV_GWB; w += 2) v += L.red[r][w][i] + L.red[r][w + 1][i];
      epilogue(P.epi[r], Rw.lo + i, v);
    }
  }
}

template <typename TD, int KB, int R>
static void gather_b(const MvInst* inst, const MvRef* rmap, int nr, int gwb, int step, hipStream_t s) {
  if (gwb == 8)
    hipLaunchKernelGGL((k_mv_gather_b<TD, KB, R, 8>), dim3(nr), dim3(64 * 8), 0, s, inst, rmap, step);
  else
    hipLaunchKernelGGL((k_mv_gather_b<TD, KB, R, MV_GWB>), dim3(nr), dim3(64 * MV_GWB), 0, s, inst, rmap, step);
}

template <int KB, int R>
static void batch_t(const MvInst* inst, const MvRef* wmap, int nw, const MvRef* rmap, int nr, bool dense_f32,
                    int gwb, int step, hipStream_t s) {
  // tiles of project_width(KB) columns into KB-wide partial slots
  constexpr int PK = project_width(KB);
  if (nw > 0)
    hipLaunchKernelGGL((k_mv_project_b<PK, R, KB>), dim3((nw + 3) / 4), dim3(256), 0, s, inst, wmap, nw, step);
  if (nr > 0) {
    if (dense_f32)
      gather_b<float, KB, R>(inst, rmap, nr, gwb, step, s);
    else
      gather_b<double, KB, R>(inst, rmap, nr, gwb, step, s);
  }
}

template <int KB>
static hipError_t batch_r(const MvInst* inst, const MvRef* wmap, int nw, const MvRef* rmap, int nr, bool dense_f32,
                          int rmax, int gwb, int step, hipStream_t s) {
  if (rmax == 1)
    batch_t<KB, 1>(inst, wmap, nw, rmap, nr, dense_f32, gwb, step, s);
  else if (rmax == 2)
    batch_t<KB, 2>(inst, wmap, nw, rmap, nr, dense_f32, gwb, step, s);
  else if (rmax == 4 && KB <= 16)
    batch_t<KB, (KB <= 16 ? 4 : 2)>(inst, wmap, nw, rmap, nr, dense_f32, gwb, step, s);
  else
    return hipErrorInvalidValue;
  return hipSuccess;
}

int mv_batch_rmax(int kb) { return kb <= 16 ? 4 : 2; }

hipError_t mv_batch_launch(const MvInst* inst, const MvRef* wmap, int nw, const MvRef* rmap, int nr, int kb,
                           bool dense_f32, int rmax, int gwb, int step, hipStream_t s) {
  if (gwb != MV_GWB && gwb != 8) return hipErrorInvalidValue;
  hipError_t e;
  if (kb == 8)
    e = batch_r<8>(inst, wmap, nw, rmap, nr, dense_f32, rmax, gwb, step, s);
  else if (kb == 16)
    e = batch_r<16>(inst, wmap, nw, rmap, nr, dense_f32, rmax, gwb, step, s);
  else if (kb == 32)
    e = batch_r<32>(inst, wmap, nw, rmap, nr, dense_f32, rmax, gwb, step, s);
  else
    return hipErrorInvalidValue;
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

__global__ void k_convert_f32(const double* in, float* out, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) out[i] = (float)in[i];
}

// FP64 -> BF16, rounded to nearest even (finite inputs)
__global__ void k_convert_bf16(const double* in, uint16_t* out, size_t n) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t stride = (size_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) {
    const uint32_t u = __float_as_uint((float)in[i]);
    out[i] = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
  }
}

hipError_t launch_convert_bf16(const double* in, uint16_t* out, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_convert_bf16, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_convert_f32(const double* in, float* out, size_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  size_t blocks = std::min<size_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_convert_f32, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

}  // namespace hl
