// Descriptors of the per-step H-matrix-vector product (mv.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hl {

constexpr int MV_KP = 32;     // partial stride (>= largest rank)
constexpr int MV_SEG = 1024;  // rows per projection segment

// One wavefront: partial[seg][p] = sum_{j in [r0, r1)} V[j + ld p] x[xoff + j], p < k.
struct MvSeg {
  int32_t r0, r1, k, ld, xoff, pad;
  const void* V;
};

// A leaf seen from one leaf cluster rho: dense block rows of rho (ptr at row
// rho.lo of the leaf, ld rows, n cols, x offset xoff) or the rows of U for
// rho (ptr at that row, ld, rank k, projection segments [sbeg, sbeg + nseg)).
struct MvEntry {
  int32_t kind;   // 0 dense, 1 low rank
  int32_t n, xoff, k, sbeg, nseg, ld, pad;
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
  const MvEntry* ents;
  const MvRow* rows;
  int32_t nseg, nrows;
  int32_t dense_f32, lr_f32;
};

hipError_t mv_launch(const MvDev& M, const double* x, double* partial, const MvEpi& epi, hipStream_t s);
// the two kernels of mv_launch separately (timing)
hipError_t project_launch(const MvDev& M, const double* x, double* partial, hipStream_t s);
hipError_t gather_launch(const MvDev& M, const double* x, const double* partial, const MvEpi& epi, hipStream_t s);
hipError_t launch_convert_f32(const double* in, float* out, size_t n, hipStream_t s);

}  // namespace hl
