// Descriptors of the per-step H-matrix-vector product (mv.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hl {

constexpr int MV_KP = 32;     // partial stride (>= largest rank)
constexpr int MV_SMALL = 1024;   // leaves with more rows are split over a whole projection block

// Projection of one low-rank leaf: t[tb][p] = sum_{j < n} V[j + ld p] x[xoff + j], p < k.
struct MvSeg {
  int32_t n, k, ld, xoff;
  int32_t tb;       // slot of the leaf's final projection
  int32_t pad;
  const void* V;
};

// A projection block (1024 threads = 16 wavefronts): `count` small leaves,
// one wavefront each, or one large leaf (big = 1) split over the 16
// wavefronts and reduced in LDS.
struct MvProjBlock {
  int32_t first, count, big, pad;
};

// A leaf seen from one leaf cluster rho: dense block rows of rho (ptr at row
// rho.lo of the leaf, ld rows, n cols, x offset xoff) or the rows of U for
// rho (ptr at that row, ld, rank k, projection slot tb).
struct MvEntry {
  int32_t kind;   // 0 dense, 1 low rank
  int32_t n, xoff, k, tb, pad, ld, pad2;
  const void* ptr;
};

struct MvRow {
  int32_t lo, hi, ebeg, eend;
};

enum { MV_EPI_PLAIN = 0, MV_EPI_RHS = 1, MV_EPI_RESID = 2, MV_EPI_ADD = 3 };

struct MvEpi {
  int32_t kind, pad;
  double hdt, cg;
  const double* u;   // RHS: u;  RESID: x
  const double* g;   // RHS forcing profile or nullptr
  const double* b;   // RESID: b
  double* y;
};

struct MvDev {
  const MvSeg* segs;
  const MvProjBlock* pblk;
  const MvEntry* ents;
  const MvRow* rows;
  double* tb;          // projections t_b, MV_KP per low-rank leaf
  int32_t npblk, nrows;
  int32_t dense_f32, lr_f32;
};

hipError_t mv_launch(const MvDev& M, const double* x, double* partial, const MvEpi& epi, hipStream_t s);
// the two kernels of mv_launch separately (timing)
hipError_t project_launch(const MvDev& M, const double* x, double* partial, hipStream_t s);
hipError_t gather_launch(const MvDev& M, const double* x, const double* partial, const MvEpi& epi, hipStream_t s);
hipError_t launch_convert_f32(const double* in, float* out, size_t n, hipStream_t s);

}  // namespace hl
