// Descriptors of the per-step H-matrix-vector product (mv.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hl {

constexpr int MV_PMAX = 32;   // at most this many projection tiles (partials) per low-rank leaf
constexpr int MV_EMAX = 128;  // entries staged in LDS per gather round
constexpr int MV_DCOLS = 16;  // columns per dense gather entry (a dense leaf is split into such pieces)

// One wavefront of the projection: rows [r0, r0 + n) and columns
// [col0, col0 + k) of the V factor of a low-rank leaf (V column-major with
// leading dimension ld; the pointer is at row r0 of column col0).  The
// wavefront writes the k partial sums sum_j V[j, col0 + p] x[xoff + j] to
// slot `slot` of the partial buffer (stride kb doubles per slot), at
// columns col0 .. col0 + k - 1.  A tile is project_width(kb) columns wide:
// a row range of a leaf of rank k takes ceil(k / width) tiles.
// columns of one projection tile for a plan of rank bucket kb
constexpr int project_width(int kb) { return kb <= 8 ? kb : (kb == 16 ? 8 : 16); }

// storage formats of a low-rank factor read by the products
enum { MV_FMT_F64 = 0, MV_FMT_F32 = 1, MV_FMT_BF16 = 2 };

struct MvTile {
  int32_t n, k, ld, xoff;
  int32_t slot, f32;   // storage format of V (MV_FMT_*)
  int32_t col0, pad;
  const void* V;       // row r0, column col0
};

// A leaf seen from one leaf cluster rho.  Dense: block rows of rho (ptr at
// row rho.lo of the leaf, leading dimension ld, n columns, x offset xoff).
// Low rank: rows of U for rho (ptr at that row, ld, rank k); its projection
// t = V^T x is the sum of np partials starting at slot `slot`.
struct MvEntry {
  int32_t kind;   // 0 dense, 1 low rank (FP64 U), 2 low rank (FP32 U), 3 low rank (BF16 U)
  int32_t n;      // dense: columns; low rank: number of partials
  int32_t xoff, k, slot, pad, ld, pad2;
  const void* ptr;
};

struct MvRow {
  int32_t lo, hi, ebeg, eend;
};

// Epilogues of the gather (v = the product's row value, r = the row):
//   PLAIN: y = v
//   RHS:   y = u + hdt v + cg g            (right side (I + dt/2 G) u + forcing)
//   RESID: y = b - (u - hdt v)             (residual of M x = b, x in u)
//   ADD:   y = u + v                       (refinement update)
//   AXPY:  y = hdt v + cg g                (g may be null)
//   CNRES: y = 2 u + cg g - (b - hdt v)    (residual of M w = 2 u + cg g, w in b)
//   NEXT:  y = b + v - u                   (u^{n+1} = w - u^n after the last update)
//   SUB:   y = v - u
// y may alias u or b: every row is read and written by the same thread.
enum {
  MV_EPI_PLAIN = 0, MV_EPI_RHS = 1, MV_EPI_RESID = 2, MV_EPI_ADD = 3,
  MV_EPI_AXPY = 4, MV_EPI_CNRES = 5, MV_EPI_NEXT = 6, MV_EPI_SUB = 7
};

struct MvEpi {
  int32_t kind, pad;
  double hdt, cg;
  const double* u;
  const double* g;   // forcing profile or nullptr
  const double* b;
  double* y;
};

struct MvDev {
  const MvTile* tiles;
  const MvEntry* ents;
  const MvRow* rows;
  double* part;        // projection partials, kb doubles per slot
  int32_t ntiles, nrows;
  int32_t kb;          // rank bucket of the matrix: 8, 16 or 32 (leaves above it are split into kb-column chunks)
  int32_t dense_f32;   // dense leaves stored in FP32 (else FP64)
  int32_t gw, gwb;     // wavefronts per gather workgroup: single-problem and batched launches (4 or 8)
};

// One problem of a batched product: its plan and nr <= MV_RMAX members
// (right-hand sides of the same operator), each with its input, partial
// buffer, epilogue and step limit (the member takes part in steps
// 0 .. steps-1 of the launching loop).
constexpr int MV_RMAX = 4;
struct MvInst {
  MvDev dev;
  int32_t nr, pad;
  int32_t steps[MV_RMAX];
  const double* x[MV_RMAX];
  double* part[MV_RMAX];
  MvEpi epi[MV_RMAX];
};

// Work item of a batched product: problem `inst` and the device address of
// its MvTile (projection) or MvRow (gather).
struct MvRef {
  int32_t inst, pad;
  const void* p;
};

hipError_t mv_launch(const MvDev& M, const double* x, const MvEpi& epi, hipStream_t s);
// Batched product over problems of one rank bucket kb, dense precision,
// member bound rmax (1, 2 or mv_batch_rmax(kb); every problem of the launch
// has nr <= rmax) and gather width gwb (4 or 8 wavefronts): wmap[w] names the tile of projection wavefront w (nw of
// them), rmap[b] the leaf cluster of gather workgroup b (nr of them).
// Members with steps <= step sit out.
hipError_t mv_batch_launch(const MvInst* inst, const MvRef* wmap, int nw, const MvRef* rmap, int nr, int kb,
                           bool dense_f32, int rmax, int gwb, int step, hipStream_t s);
// largest member count of a batched problem with rank bucket kb
int mv_batch_rmax(int kb);
// the two kernels of mv_launch separately; non-null events are attached to
// the dispatch (start, stop) for timing
hipError_t project_launch(const MvDev& M, const double* x, hipStream_t s, hipEvent_t e0 = nullptr,
                          hipEvent_t e1 = nullptr);
hipError_t gather_launch(const MvDev& M, const double* x, const MvEpi& epi, hipStream_t s,
                         hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// rows of V one projection wavefront covers per pass (64 lanes x rows per
// lane); narrow: FP32 or BF16 storage
int project_rows_per_pass(int kb, bool narrow);
hipError_t launch_convert_f32(const double* in, float* out, size_t n, hipStream_t s);
hipError_t launch_convert_bf16(const double* in, uint16_t* out, size_t n, hipStream_t s);

}  // namespace hl
