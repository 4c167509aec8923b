// Work descriptors consumed by the HIP kernels.  Plain structs with raw
// device pointers; the host fills them and copies them to the device once
// per plan.
#pragma once

#include <cstdint>

#include "hl_internal.h"

namespace hl {

constexpr int KMAX = 64;       // widest concatenation handled by one rounded addition
// Rounded additions below this truncation tolerance carry double-double
// parts through the Gram products (a Gram in FP64 resolves the truncation
// error only down to about sqrt(eps) = 1.5e-8 of the sum: at 1e-9 the
// measured per-block error was 3e-9); without them the LDS of the fused
// kernel takes concatenations of KMAX columns, with them 48.
constexpr double RADD_DD_TOL = 1e-8;
constexpr bool radd_dd(double tol) { return tol < RADD_DD_TOL; }
constexpr int fused_width(double tol) { return radd_dd(tol) ? 48 : KMAX; }
constexpr int LEAFMAX = 64;    // largest leaf cluster
constexpr int GRAM_CHUNK = 512;  // rows per Gram / expand work item

// Leaf-cluster lists of the block tree on the device.
struct DevLists {
  const int32_t* rowptr;
  const int32_t* rowidx;
  const int32_t* colptr;
  const int32_t* colidx;
  const int32_t* lc_lo;   // per leaf-cluster position: first index
  const int32_t* lc_hi;   // one past the last index
};

// Y = op(B_sub) X for the sub-block B_sub = leaves [lbeg, lend) of a matrix,
// covering rows [rlo, rhi) and cols [clo, chi).  op = identity (trans = 0):
// X has rows indexed from clo, Y from rlo.  trans = 1: X rows from rlo,
// Y rows from clo.  kx columns (device int, or kxcap when kx == nullptr).
// dl: the leaf-cluster lists of the matrix's block tree (jobs of one launch
// may belong to different problems).
struct ApplyJob {
  DevLists dl;
  const LeafDesc* L;
  const int32_t* rank;
  int32_t lbeg, lend;
  int32_t rlo, rhi, clo, chi;
  int32_t trans;
  int32_t ldx, ldy, kxcap;
  const double* X;
  const int32_t* kx;
  double* Y;
  double* T;        // projection slots, (leaf - lbeg) * tstride doubles each
  int32_t tstride;
  int32_t pad;
};

struct ProjItem { int32_t job, leaf; };
struct GatherItem { int32_t job, lpos; };

// P (m x n, ld ldp) = A (m x k, ld lda) * B (k x n, ld ldb), all <= 64.
struct DProdItem {
  const double* A;
  const double* B;
  double* P;
  int32_t lda, ldb, ldp, m, k, n;
};

// One update term of a target block:
//   C[ro:ro+mr, co:co+nc] += sign * U W^T     (low rank, k columns), or
//   C[ro:ro+mr, co:co+nc] += sign * P          (dense, P in U with ld ldu).
// U points at the row of the factor that corresponds to region row 0,
// W at the row that corresponds to region column 0.
// An update term over rows [ro, ro + mr) x columns [co, co + nc) of a target:
//   dense = 0: sign * U W^T, U mr x k (ld ldu), W nc x k (ld ldw), k = *k or kfix
//   dense = 1: sign * P, P mr x nc (U, ld ldu)
//   dense = 2: sign * A B, A mr x kfix (U, ld ldu), B kfix x nc (W, ld ldw)
// klim > 0 (dense = 0): the term is columns [kofs, kofs + klim) of a wider
// low-rank term (U and W already point at column kofs): its rank is
// clamp(k - kofs, 0, klim).
struct Term {
  int32_t dense;
  int32_t ro, mr, co, nc;
  int32_t ldu, ldw, kfix;
  const double* U;
  const double* W;
  const int32_t* k;   // rank (device) or nullptr => kfix
  double sign;
  int32_t kofs, klim;
};

// Dense target: D (m x n, ld ldd) += sum of terms [tbeg, tbeg + tcount).
struct DFlushItem {
  double* D;
  int32_t ldd, m, n, tbeg, tcount;
  int32_t pad;
};

// Low-rank target: C = U V^T (U m x kcap, V n x kcap, rank *rank) is
// replaced by the truncated SVD of C + sum of its terms (rounded addition).
struct LFlushTarget {
  double* U;
  double* V;
  int32_t* rank;       // nullptr => the target starts empty
  int32_t m, n, kcap, Kcap;
  int32_t tbeg, tcount;
  int32_t nchA, nchB;  // Gram chunks on the U side / V side
  double* ws;          // workspace of this target
  int32_t* info;       // [0] old rank, [1] new rank, [2] overflow
  int32_t* overflow;   // global overflow counter
  int32_t borth;       // 1: every term's right factor is a set of unit columns, disjoint
                       // across the terms (a dense block split by columns), so the
                       // concatenated B of an empty target has B^T B = I
  int32_t pad;
};

struct ChunkItem { int32_t tgt, side, r0, r1, chunk, pad; };

// Copy of a leaf between two matrices with the same structure.
struct CopyItem {
  const double* A;
  const double* B;
  double* dA;
  double* dB;
  const int32_t* rank;
  int32_t* drank;
  int32_t m, n, kcap, dense;
  double scale;        // applied to A (dense block or U)
  int32_t add_identity;  // dense diagonal leaf: add the identity after scaling
  int32_t expand;        // destination dense, source low rank: dA = scale * U V^T
  double* zA;            // move: the dense source (zeroed after the copy) or nullptr
  int32_t* zrank;        // move: the low-rank source's rank (set to 0) or nullptr
};

// Leaf factorisation: LU in place (no pivoting) and the inverses of the
// unit-lower and upper factors.
// Dense diagonal block of at most 2 x 2 leaf tiles, n = m1 + m2 <= LUINV_N
// (m2 = 0: a single leaf): LU without pivoting and the inverses of both
// factors.  Tiles are column-major with leading dimension = their row count.
constexpr int LUINV_N = 128;
struct LuInvItem {
  const double* A11;
  const double* A12;
  const double* A21;
  const double* A22;
  double* L11;   // blocks of L^{-1} (L12 = 0)
  double* L21;
  double* L22;
  double* U11;   // blocks of U^{-1} (U21 = 0)
  double* U12;
  double* U22;
  int32_t m1, m2;
};

struct GetrfItem {
  double* LU;
  double* Li;
  double* Ui;
  int32_t m, pad;
};

// Problem data needed on the device for assembly.
struct ProblemDev {
  int32_t dim, n, N;
  double h, a, b0, b1, c, s, lam, C, r0;
  int32_t kernel, pad;   // hlevy_kernel
  double eps2;           // Gaussian: nu(r) = C exp(-eps2 r^2)
  double lam_neg;        // asymmetric tempered kernel: rate of the jumps y < 0 (lam: y > 0)
  // variable-order kernel: per distinct jump index its value, kernel
  // constant and five quadrature constants; per cluster position (row) the
  // index of its value
  const double* var_s;
  const double* var_C;
  const double* var_cst;
  const int32_t* var_row;
  int32_t nvar, pad2;
};

}  // namespace hl
