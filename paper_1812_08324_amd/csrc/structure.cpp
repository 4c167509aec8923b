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

// Two centres of Lloyd's iteration (Sec. 5.4: recursive K-means with two
// clusters) over the points [lo, hi) of a 2D cluster, on their integer grid
// coordinates.  Centre A = SA / nA.  A point goes to B only when strictly
// nearer: |nB p - SB|^2 nA^2 < |nA p - SA|^2 nB^2, compared exactly (the
// factors stay below 2^115 for n <= 8192 and N <= 2^22).  Returns the side
// of every point (true: B) after at most 64 assignment passes, stopping when
// no point moves; a pass that would empty a side is discarded.
std::vector<char> kmeans2(const Structure& s, int lo, int hi) {
  using i128 = __int128;
  const int cnt = hi - lo;
  std::vector<int64_t> g(2 * (size_t)cnt);
  for (int i = 0; i < cnt; ++i) {
    g[2 * i] = s.lat[lo + i] / s.n;
    g[2 * i + 1] = s.lat[lo + i] % s.n;
  }
  int64_t mn[2] = {g[0], g[1]}, mx[2] = {g[0], g[1]};
  for (int i = 1; i < cnt; ++i)
    for (int a = 0; a < 2; ++a) {
      mn[a] = std::min(mn[a], g[2 * i + a]);
      mx[a] = std::max(mx[a], g[2 * i + a]);
    }
  const int ax = (mx[1] - mn[1] > mx[0] - mn[0]) ? 1 : 0;
  int ia = -1, ib = -1;
  for (int i = 0; i < cnt; ++i) {
    if (ia < 0 && g[2 * i + ax] == mn[ax]) ia = i;
    if (ib < 0 && g[2 * i + ax] == mx[ax]) ib = i;
  }
  int64_t SA[2] = {g[2 * ia], g[2 * ia + 1]}, SB[2] = {g[2 * ib], g[2 * ib + 1]};
  int64_t nA = 1, nB = 1;
  std::vector<char> prev, cur(cnt);
  for (int it = 0; it < 64; ++it) {
    int64_t inB = 0;
    for (int i = 0; i < cnt; ++i) {
      i128 dA = 0, dB = 0;
      for (int a = 0; a < 2; ++a) {
        const i128 ea = (i128)nA * g[2 * i + a] - SA[a], eb = (i128)nB * g[2 * i + a] - SB[a];
        dA += ea * ea;
        dB += eb * eb;
      }
      cur[i] = dB * ((i128)nA * nA) < dA * ((i128)nB * nB);
      inB += cur[i];
    }
    if (cur == prev) break;
    if (inB == 0 || inB == cnt) break;   // keeps prev (the first pass never empties a side)
    prev = cur;
    SA[0] = SA[1] = SB[0] = SB[1] = 0;
    nA = nB = 0;
    for (int i = 0; i < cnt; ++i) {
      int64_t* S = cur[i] ? SB : SA;
      S[0] += g[2 * i];
      S[1] += g[2 * i + 1];
      (cur[i] ? nB : nA) += 1;
    }
  }
  return prev;
}

// Split cluster `id` into two children, keeping the order inside halves.
// BISECT: 1D halves the index range (floor(n/2), n - floor(n/2)); 2D
// bisects the longest side of the bounding box at its midpoint (ties: first
// axis).  KMEANS (2D): the two clusters of kmeans2.
void split(Structure& s, int id) {
  Cluster c = s.cl[id];
  int nl;
  if (s.dim == 1) {
    nl = (c.hi - c.lo) / 2;
  } else {
    std::vector<char> side;
    if (s.cluster == HLEVY_CLUSTER_KMEANS) side = kmeans2(s, c.lo, c.hi);
    if (side.empty()) {
      int ax = (c.bmax[1] - c.bmin[1] > c.bmax[0] - c.bmin[0]) ? 1 : 0;
      double mid = 0.5 * (c.bmin[ax] + c.bmax[ax]);
      side.resize(c.hi - c.lo);
      for (int i = c.lo; i < c.hi; ++i) side[i - c.lo] = !(s.pts[(size_t)i * 2 + ax] < mid);
    }
    std::vector<int32_t> left, right, ll, lr;
    std::vector<double> pl, pr;
    for (int i = c.lo; i < c.hi; ++i) {
      const bool r = side[i - c.lo];
      (r ? right : left).push_back(s.perm[i]);
      (r ? lr : ll).push_back(s.lat[i]);
      std::vector<double>& P = r ? pr : pl;
      P.push_back(s.pts[(size_t)i * 2]);
      P.push_back(s.pts[(size_t)i * 2 + 1]);
    }
    nl = (int)left.size();
    std::copy(left.begin(), left.end(), s.perm.begin() + c.lo);
    std::copy(right.begin(), right.end(), s.perm.begin() + c.lo + nl);
    std::copy(ll.begin(), ll.end(), s.lat.begin() + c.lo);
    std::copy(lr.begin(), lr.end(), s.lat.begin() + c.lo + nl);
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
  // a fixed-rank Taylor block needs at least taylor_rank rows and columns
  // (below that a dense block is both exact and smaller)
  const bool thin = s.taylor_rank > 0 && std::min(R.hi - R.lo, C.hi - C.lo) < s.taylor_rank;
  if (adm && sz <= s.nmax && r != c && !over && !thin) {
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
           p.kernel != HLEVY_KERNEL_TEMPERED_ASYM && p.kernel != HLEVY_KERNEL_VARIABLE_ORDER)
    err << "kernel must be HLEVY_KERNEL_TEMPERED, HLEVY_KERNEL_GAUSSIAN, HLEVY_KERNEL_TEMPERED_ASYM or "
           "HLEVY_KERNEL_VARIABLE_ORDER";
  else if (p.mask && p.dim != 2) err << "a mask needs dim 2";
  else if (p.kernel == HLEVY_KERNEL_VARIABLE_ORDER && !p.s_field) err << "the variable-order kernel needs s_field";
  else if (p.kernel != HLEVY_KERNEL_VARIABLE_ORDER && p.s_field)
    err << "s_field is for the variable-order kernel only";
  else if (hp.cluster != HLEVY_CLUSTER_BISECT && hp.cluster != HLEVY_CLUSTER_KMEANS)
    err << "cluster must be HLEVY_CLUSTER_BISECT or HLEVY_CLUSTER_KMEANS";
  else if (hp.cluster == HLEVY_CLUSTER_KMEANS && p.dim != 2) err << "KMEANS clustering is 2D only";
  else if (p.kernel == HLEVY_KERNEL_TEMPERED_ASYM && (!(p.lambda_neg >= 0.0) || !std::isfinite(p.lambda_neg)))
    err << "lambda_neg must be >= 0";
  else if (p.kernel != HLEVY_KERNEL_GAUSSIAN && p.kernel != HLEVY_KERNEL_VARIABLE_ORDER && !(p.s > 0.0 && p.s < 1.0))
    err << "s must lie in (0, 1)";
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
  const int64_t grid = p.dim == 1 ? (int64_t)p.n : (int64_t)p.n * p.n;
  if (grid > (int64_t)1 << 26) return "grid too large (max 2^26 points)";
  // unknowns: the grid points in grid order, or those the mask keeps
  std::vector<int32_t> kept;
  if (p.mask) {
    for (int64_t g = 0; g < grid; ++g)
      if (p.mask[g]) kept.push_back((int32_t)g);
  }
  int64_t N64 = p.mask ? (int64_t)kept.size() : grid;
  if (N64 < 2 * (int64_t)hp.leaf) return "N must be at least twice the leaf size";
  if (hp.cluster == HLEVY_CLUSTER_KMEANS && N64 > (int64_t)1 << 22) return "KMEANS clustering needs N <= 2^22";
  if (p.kernel == HLEVY_KERNEL_VARIABLE_ORDER)
    for (int64_t i = 0; i < N64; ++i)
      if (!(p.s_field[i] > 0.0 && p.s_field[i] < 1.0))
        return "s_field[" + std::to_string(i) + "] must lie in (0, 1)";

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
  s.cluster = hp.cluster;
  s.taylor_rank = hp.taylor_rank;
  const int N = s.N;
  s.perm.resize(N);
  std::iota(s.perm.begin(), s.perm.end(), 0);
  if (p.mask) s.lat = kept;
  else s.lat = s.perm;
  s.pts.resize((size_t)N * s.dim);
  if (s.dim == 1) {
    for (int i = 0; i < N; ++i) s.pts[i] = p.lo + (i + 1) * s.h;
  } else {
    for (int k = 0; k < N; ++k) {
      const int g = s.lat[k];
      s.pts[2 * (size_t)k] = p.lo + (g / s.n + 1) * s.h;
      s.pts[2 * (size_t)k + 1] = p.lo + (g % s.n + 1) * s.h;
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

  if (p.kernel == HLEVY_KERNEL_VARIABLE_ORDER) {
    // distinct jump indices, ascending; each cluster position's row
    s.var_s.assign(p.s_field, p.s_field + N);
    std::sort(s.var_s.begin(), s.var_s.end());
    s.var_s.erase(std::unique(s.var_s.begin(), s.var_s.end()), s.var_s.end());
    s.var_row.resize(N);
    for (int k = 0; k < N; ++k)
      s.var_row[k] = (int32_t)(std::lower_bound(s.var_s.begin(), s.var_s.end(), p.s_field[s.perm[k]]) -
                               s.var_s.begin());
  }
  build_block(s, 0, 0);
  number_leaves(s, 0);
  for (auto& l : s.lf) {
    if (l.kind == K_DENSE) {
      s.n_dense++;
      s.dense_entries += (int64_t)l.m * l.n;
    } else {
      s.n_lr++;
      // the ACA kernel marks used pivot rows in a bitmap of LR_ROWS_MAX bits
      // (the Taylor construction runs no ACA)
      if (hp.taylor_rank == 0 && std::max(l.m, l.n) > LR_ROWS_MAX)
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
