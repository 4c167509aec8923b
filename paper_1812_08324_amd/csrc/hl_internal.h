// Internal declarations shared by the host code and the HIP kernels of the
// H-matrix Crank-Nicolson library.  Nothing here crosses the C ABI.
#pragma once

#include <cstdint>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "hlevy.h"

namespace hl {

// ---------------------------------------------------------------------------
// Trees (App. B.1): a balanced binary cluster tree whose leaves all sit at
// the same depth, and the block tree built with the admissibility of
// eq. equ:adm on the bounding boxes of the point sets.
// ---------------------------------------------------------------------------
enum Kind : int32_t { K_H = 0, K_DENSE = 1, K_LR = 2, K_ZERO = 3 };

struct Cluster {
  int32_t lo, hi, level;
  int32_t child[2];
  double bmin[2], bmax[2];
};

struct BNode {
  int32_t r, c;      // cluster ids
  int32_t kind;      // K_H, K_DENSE or K_LR
  int32_t child[4];  // (i, j) -> child[2 i + j] for K_H
  int32_t leaf;      // leaf id for leaves, -1 for K_H
  int32_t lbeg, lend;  // DFS range of the leaves below this node
};

struct LeafInfo {
  int32_t r, c, kind;
  int32_t rlo, clo, m, n;
};

struct Structure {
  int32_t dim = 1, n = 0, N = 0, leaf = 64, depth = 0, nmax = 0;
  double lo = -1, hi = 1, h = 0, eta = 1;
  std::vector<int32_t> perm;    // cluster position -> natural index
  std::vector<int32_t> lat;     // cluster position -> grid index (1D: i; 2D: p*n + q); = perm without a mask
  // variable-order kernel: the distinct jump indices (ascending) and, per
  // cluster position, the index of its row's value among them
  std::vector<double> var_s;
  std::vector<int32_t> var_row;
  int32_t cluster = 0;          // hlevy_cluster
  int32_t taylor_rank = 0;      // > 0: admissible blocks with fewer rows or columns are dense
  std::vector<double> pts;      // coordinates in cluster order (N * dim)
  std::vector<Cluster> cl;      // cl[0] is the root
  std::vector<int32_t> leafcl;  // leaf clusters in index order
  std::vector<int32_t> leafpos; // cluster id -> position in leafcl (-1 if not a leaf)
  std::vector<BNode> bn;        // bn[0] is the root block (root, root)
  std::vector<LeafInfo> lf;     // leaves in DFS order
  // For every leaf cluster rho: leaves whose row (col) cluster contains rho,
  // ordered by column (row) start.
  std::vector<int32_t> rowptr, rowidx, colptr, colidx;
  // leaf cluster position containing index i: i -> position (size N)
  int32_t n_dense = 0, n_lr = 0;
  int64_t dense_entries = 0;
  // admissible blocks (row cluster, column cluster) not stored low rank:
  // subdivided, or dense at the leaf level (R16: ACA over the rank cap)
  std::set<std::pair<int32_t, int32_t>> split;
};

// Largest side of an admissible (low-rank) block: the ACA kernel keeps its
// used pivot rows in an LDS bitmap of this many bits.
constexpr int32_t LR_ROWS_MAX = 16384;

// Validates the descriptor and builds every host structure.  Returns an
// error message on failure (empty on success).
std::string build_structure(const hlevy_problem& p, const hlevy_hparams& hp, Structure& s,
                            const std::set<std::pair<int32_t, int32_t>>* split = nullptr);

// Sets the thread-local message hlevy_last_error() returns.
void set_last_error(const std::string& msg);

// Whether the leaf is strictly below / above the diagonal.
inline bool leaf_lower(const LeafInfo& l) { return l.clo + l.n <= l.rlo; }
inline bool leaf_upper(const LeafInfo& l) { return l.rlo + l.m <= l.clo; }

// ---------------------------------------------------------------------------
// Device-visible descriptors (plain structs, identical layout on host and
// device).
// ---------------------------------------------------------------------------
struct LeafDesc {
  int32_t kind;      // K_DENSE, K_LR or K_ZERO
  int32_t m, n;      // rows, cols
  int32_t rlo, clo;  // first row / col (cluster order)
  int32_t kcap;      // rank capacity (K_LR)
  double* A;         // dense m x n col-major (ld m) | U: m x kcap (ld m)
  double* B;         // V: n x kcap (ld n)
};

}  // namespace hl
