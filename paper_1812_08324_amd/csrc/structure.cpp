// Host-side construction of the cluster tree, the block tree and the
// per-leaf-cluster block lists (App. B.1 of Xu & Darve).
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <sstream>

#include "hl_internal.h"

namespace hl {

namespace {

void set_box(Structure& s, Cluster& c) {
  const int d = s.dim;
  for (int a = 0; a < 2; ++a) { c.bmin[a] = 0; c.bmax[a] = 0; }
  for (int a = 0; a < d; ++a) {
    double mn = INFINITY, mx = -INFINITY;
    for (int i = c.lo; i < c.hi; ++i) {
      double v = s.pts[(size_t)i * d + a];
      mn = std::min(mn, v);
      mx = std::max(mx, v);
    }
    c.bmin[a] = mn;
    c.bmax[a] = mx;
  }
}

double diam(const Structure& s, const Cluster& c) {
  double acc = 0;
  for (int a = 0; a < s.dim; ++a) acc += (c.bmax[a] - c.bmin[a]) * (c.bmax[a] - c.bmin[a]);
  return std::sqrt(acc);
}

double dist(const Structure& s, const Cluster& x, const Cluster& y) {
  double acc = 0;
  for (int a = 0; a < s.dim; ++a) {
    double g = std::max(0.0, std::max(x.bmin[a] - y.bmax[a], y.bmin[a] - x.bmax[a]));
    acc += g * g;
  }
  return std::sqrt(acc);
}

// Split cluster `id` into two children: 1D halves the index range
// (floor(n/2), n - floor(n/2)); 2D bisects the longest side of the bounding
// box at its midpoint (ties: first axis), keeping the order inside halves.
void split(Structure& s, int id) {
  Cluster c = s.cl[id];
  int nl;
  if (s.dim == 1) {
    nl = (c.hi - c.lo) / 2;
  } else {
    int ax = (c.bmax[1] - c.bmin[1] > c.bmax[0] - c.bmin[0]) ? 1 : 0;
    double mid = 0.5 * (c.bmin[ax] + c.bmax[ax]);
    std::vector<int32_t> left, right;
    std::vector<double> pl, pr;
    for (int i = c.lo; i < c.hi; ++i) {
      double v = s.pts[(size_t)i * 2 + ax];
      if (v < mid) {
        left.push_back(s.perm[i]);
        pl.push_back(s.pts[(size_t)i * 2]);
        pl.push_back(s.pts[(size_t)i * 2 + 1]);
      } else {
        right.push_back(s.perm[i]);
        pr.push_back(s.pts[(size_t)i * 2]);
        pr.push_back(s.pts[(size_t)i * 2 + 1]);
      }
    }
    nl = (int)left.size();
    std::copy(left.begin(), left.end(), s.perm.begin() + c.lo);
    std::copy(right.begin(), right.end(), s.perm.begin() + c.lo + nl);
    std::copy(pl.begin(), pl.end(), s.pts.begin() + (size_t)c.lo * 2);
    std::copy(pr.begin(), pr.end(), s.pts.begin() + (size_t)(c.lo + nl) * 2);
  }
  Cluster a{}, b{};
  a.lo = c.lo; a.hi = c.lo + nl; a.level = c.level + 1; a.child[0] = a.child[1] = -1;
  b.lo = c.lo + nl; b.hi = c.hi; b.level = c.level + 1; b.child[0] = b.child[1] = -1;
  set_box(s, a);
  set_box(s, b);
  int ia = (int)s.cl.size();
  s.cl.push_back(a);
  s.cl.push_back(b);
  s.cl[id].child[0] = ia;
  s.cl[id].child[1] = ia + 1;
}

int build_block(Structure& s, int r, int c) {
  int id = (int)s.bn.size();
  s.bn.push_back(BNode{});
  BNode b{};
  b.r = r; b.c = c; b.leaf = -1;
  for (int q = 0; q < 4; ++q) b.child[q] = -1;
  const Cluster& R = s.cl[r];
  const Cluster& C = s.cl[c];
  bool adm = std::min(diam(s, R), diam(s, C)) <= s.eta * dist(s, R, C);
  int sz = std::max(R.hi - R.lo, C.hi - C.lo);
  // an admissible block whose compression needed more than the rank
  // capacity is subdivided (its children are admissible too), or kept
  // dense when its clusters are leaves
  const bool over = s.split.count({r, c}) > 0;
  if (adm && sz <= s.nmax && r != c && !over) {
    b.kind = K_LR;
  } else if (R.child[0] < 0 || C.child[0] < 0) {
    b.kind = K_DENSE;
  } else {
    b.kind = K_H;
  }
  s.bn[id] = b;
  if (b.kind == K_H) {
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) {
        int ch = build_block(s, s.cl[r].child[i], s.cl[c].child[j]);
        s.bn[id].child[2 * i + j] = ch;
      }
  }
  return id;
}

void number_leaves(Structure& s, int id) {
  BNode& b = s.bn[id];
  b.lbeg = (int)s.lf.size();
  if (b.kind == K_H) {
    for (int q = 0; q < 4; ++q) number_leaves(s, s.bn[id].child[q]);
  } else {
    const Cluster& R = s.cl[b.r];
    const Cluster& C = s.cl[b.c];
    LeafInfo li{b.r, b.c, b.kind, R.lo, C.lo, R.hi - R.lo, C.hi - C.lo};
    s.bn[id].leaf = (int)s.lf.size();
    s.lf.push_back(li);
  }
  s.bn[id].lend = (int)s.lf.size();
}

}  // namespace

std::string build_structure(const hlevy_problem& p, const hlevy_hparams& hp, Structure& s,
                            const std::set<std::pair<int32_t, int32_t>>* overcap) {
  std::ostringstream err;
  if (p.dim != 1 && p.dim != 2) err << "dim must be 1 or 2";
  else if (p.n < 2) err << "n must be >= 2";
  else if (!(p.hi > p.lo) || !std::isfinite(p.lo) || !std::isfinite(p.hi)) err << "need lo < hi (finite)";
  else if (p.kernel != HLEVY_KERNEL_TEMPERED && p.kernel != HLEVY_KERNEL_GAUSSIAN &&
           p.kernel != HLEVY_KERNEL_TEMPERED_ASYM)
    err << "kernel must be HLEVY_KERNEL_TEMPERED, HLEVY_KERNEL_GAUSSIAN or HLEVY_KERNEL_TEMPERED_ASYM";
  else if (p.kernel == HLEVY_KERNEL_TEMPERED_ASYM && p.dim != 1) err << "the asymmetric kernel is 1D only";
  else if (p.kernel == HLEVY_KERNEL_TEMPERED_ASYM && (!(p.lambda_neg >= 0.0) || !std::isfinite(p.lambda_neg)))
    err << "lambda_neg must be >= 0";
  else if (p.kernel != HLEVY_KERNEL_GAUSSIAN && !(p.s > 0.0 && p.s < 1.0)) err << "s must lie in (0, 1)";
  else if (p.kernel == HLEVY_KERNEL_GAUSSIAN && (!(p.eps2 > 0.0) || !std::isfinite(p.eps2)))
    err << "eps2 must be > 0 for the Gaussian kernel";
  else if (!(p.a >= 0.0) || !std::isfinite(p.a)) err << "a must be >= 0";
  else if (!(p.c <= 0.0) || !std::isfinite(p.c)) err << "c must be <= 0";
  else if (p.kernel != HLEVY_KERNEL_GAUSSIAN && (!(p.lambda >= 0.0) || !std::isfinite(p.lambda)))
    err << "lambda must be >= 0";
  else if (!std::isfinite(p.b[0]) || !std::isfinite(p.b[1]) || !std::isfinite(p.C)) err << "non-finite drift or C";
  else if (p.kernel != HLEVY_KERNEL_GAUSSIAN && (!(p.r0 > 0.0) || !std::isfinite(p.r0))) err << "r0 must be > 0";
  else if (p.kernel != HLEVY_KERNEL_GAUSSIAN && !(p.r0 < p.hi - p.lo)) err << "r0 must be smaller than the domain";
  else if (hp.leaf < 16 || hp.leaf > 64) err << "leaf must be in [16, 64]";
  else if (!(hp.eta > 0.0)) err << "eta must be > 0";
  else if (hp.n_block < 1) err << "n_block must be >= 1";
  else if (!(hp.aca_tol > 0.0 && hp.aca_tol < 1.0)) err << "aca_tol must be in (0, 1)";
  else if (hp.max_rank < 4 || hp.max_rank > 32) err << "max_rank must be in [4, 32]";
  else if (hp.gather_waves != 0 && hp.gather_waves != 4 && hp.gather_waves != 8) err << "gather_waves must be 0, 4 or 8";
  else if (hp.rank_bucket != 0 && hp.rank_bucket != 8 && hp.rank_bucket != 16 && hp.rank_bucket != 32)
    err << "rank_bucket must be 0, 8, 16 or 32";
  else if (hp.strict_rank_cap != 0 && hp.strict_rank_cap != 1) err << "strict_rank_cap must be 0 or 1";
  else if (hp.taylor_rank < 0 || hp.taylor_rank > hp.max_rank) err << "taylor_rank must be in [0, max_rank]";
  else if (hp.taylor_rank > 0 && p.kernel != HLEVY_KERNEL_GAUSSIAN)
    err << "taylor_rank needs the Gaussian kernel (the Taylor factors are those of exp(-eps2 |y|^2))";
  else if (hp.taylor_rank == 0 && p.kernel == HLEVY_KERNEL_GAUSSIAN)
    err << "the Gaussian kernel needs taylor_rank > 0 (partially pivoted ACA misses parts of its blocks)";
  if (!err.str().empty()) return err.str();
  int64_t N64 = p.dim == 1 ? (int64_t)p.n : (int64_t)p.n * p.n;
  if (N64 > (int64_t)1 << 26) return "N too large (max 2^26)";
  if (N64 < 2 * (int64_t)hp.leaf) return "N must be at least twice the leaf size";

  s = Structure{};
  if (overcap) s.split = *overcap;
  s.dim = p.dim;
  s.n = p.n;
  s.N = (int32_t)N64;
  s.leaf = hp.leaf;
  s.lo = p.lo;
  s.hi = p.hi;
  s.h = (p.hi - p.lo) / (p.n + 1);
  s.eta = hp.eta;
  s.nmax = (int32_t)((N64 + hp.n_block - 1) / hp.n_block);
  const int N = s.N;
  s.perm.resize(N);
  std::iota(s.perm.begin(), s.perm.end(), 0);
  s.pts.resize((size_t)N * s.dim);
  if (s.dim == 1) {
    for (int i = 0; i < N; ++i) s.pts[i] = p.lo + (i + 1) * s.h;
  } else {
    for (int i = 0; i < s.n; ++i)
      for (int j = 0; j < s.n; ++j) {
        size_t k = (size_t)i * s.n + j;
        s.pts[2 * k] = p.lo + (i + 1) * s.h;
        s.pts[2 * k + 1] = p.lo + (j + 1) * s.h;
      }
  }
  Cluster root{};
  root.lo = 0; root.hi = N; root.level = 0; root.child[0] = root.child[1] = -1;
  set_box(s, root);
  s.cl.push_back(root);
  // split level by level until every cluster has at most `leaf` points;
  // all leaves end at the same depth
  std::vector<int> frontier{0};
  for (;;) {
    int mx = 0, mn = N;
    for (int id : frontier) {
      int sz = s.cl[id].hi - s.cl[id].lo;
      mx = std::max(mx, sz);
      mn = std::min(mn, sz);
    }
    if (mx <= s.leaf) break;
    if (mn < 2) return "cluster tree cannot be balanced (cluster with < 2 points)";
    std::vector<int> next;
    for (int id : frontier) {
      split(s, id);
      next.push_back(s.cl[id].child[0]);
      next.push_back(s.cl[id].child[1]);
    }
    frontier.swap(next);
    s.depth++;
  }
  // leaf clusters in index order (frontier is already in index order)
  s.leafcl = frontier;
  s.leafpos.assign(s.cl.size(), -1);
  for (size_t q = 0; q < frontier.size(); ++q) s.leafpos[frontier[q]] = (int)q;
  for (size_t q = 0; q < frontier.size(); ++q)
    if (s.cl[frontier[q]].hi - s.cl[frontier[q]].lo < 1) return "empty leaf cluster";

  build_block(s, 0, 0);
  number_leaves(s, 0);
  for (auto& l : s.lf) {
    if (l.kind == K_DENSE) {
      s.n_dense++;
      s.dense_entries += (int64_t)l.m * l.n;
    } else {
      s.n_lr++;
      // the ACA kernel marks used pivot rows in a bitmap of LR_ROWS_MAX bits
      if (std::max(l.m, l.n) > LR_ROWS_MAX)
        return "low-rank blocks are limited to " + std::to_string(LR_ROWS_MAX) + " rows (raise n_block)";
    }
  }
  // per-leaf-cluster lists
  const int P = (int)s.leafcl.size();
  std::vector<int32_t> first_leafpos(N);
  for (int q = 0; q < P; ++q) {
    const Cluster& c = s.cl[s.leafcl[q]];
    for (int i = c.lo; i < c.hi; ++i) first_leafpos[i] = q;
  }
  std::vector<std::vector<std::pair<int, int>>> rows(P), cols(P);
  for (int l = 0; l < (int)s.lf.size(); ++l) {
    const LeafInfo& L = s.lf[l];
    int q0 = first_leafpos[L.rlo], q1 = first_leafpos[L.rlo + L.m - 1];
    for (int q = q0; q <= q1; ++q) rows[q].push_back({L.clo, l});
    q0 = first_leafpos[L.clo];
    q1 = first_leafpos[L.clo + L.n - 1];
    for (int q = q0; q <= q1; ++q) cols[q].push_back({L.rlo, l});
  }
  s.rowptr.assign(P + 1, 0);
  s.colptr.assign(P + 1, 0);
  for (int q = 0; q < P; ++q) {
    std::sort(rows[q].begin(), rows[q].end());
    std::sort(cols[q].begin(), cols[q].end());
    s.rowptr[q + 1] = s.rowptr[q] + (int)rows[q].size();
    s.colptr[q + 1] = s.colptr[q] + (int)cols[q].size();
    for (auto& e : rows[q]) s.rowidx.push_back(e.second);
    for (auto& e : cols[q]) s.colidx.push_back(e.second);
  }
  return "";
}

}  // namespace hl
