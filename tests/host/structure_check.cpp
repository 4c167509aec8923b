// Host check of the tree and block-structure builder, built with AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py (no device
// code, no GPU).  For a grid of valid descriptors it builds the structure and
// checks its invariants: the permutation is one, every cluster range nests in
// its parent's, the leaves tile the N x N index square exactly once, and the
// per-leaf-cluster row and column lists name exactly the leaves that touch each
// leaf cluster.  It then subdivides a seeded selection of admissible blocks
// (the rank-cap path) and checks the tiling again; builds masked 2D domains
// (L-shape, random, disc) with bisection and 2-means trees, variable-order
// fields and Taylor blocks and checks their maps; and feeds invalid
// descriptors that must be rejected.  Exit status 0 when every check holds.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "hl_internal.h"

namespace {

int failures = 0;

void check(bool ok, const char* what, const hlevy_problem& p, const hlevy_hparams& hp) {
  if (ok) return;
  ++failures;
  std::fprintf(stderr, "FAIL %s: dim %d n %d leaf %d eta %g n_block %d\n", what, p.dim, p.n, hp.leaf, hp.eta,
               hp.n_block);
}

hlevy_problem problem(int dim, int n) {
  hlevy_problem p{};
  p.dim = dim;
  p.n = n;
  p.lo = -1.0;
  p.hi = 1.0;
  p.s = 0.5;
  p.C = -1.0;
  p.r0 = 0.2;
  p.kernel = HLEVY_KERNEL_TEMPERED;
  return p;
}

hlevy_hparams hparams(int leaf, double eta, int n_block) {
  hlevy_hparams h{};
  h.leaf = leaf;
  h.eta = eta;
  h.n_block = n_block;
  h.aca_tol = 1e-10;
  h.max_rank = 16;
  return h;
}

void invariants(const hl::Structure& S, const hlevy_problem& p, const hlevy_hparams& hp) {
  const int N = S.N;
  std::vector<int> seen(N, 0);
  for (int v : S.perm)
    if (v >= 0 && v < N) seen[v]++;
  bool perm_ok = (int)S.perm.size() == N;
  for (int c : seen) perm_ok = perm_ok && c == 1;
  check(perm_ok, "perm is a permutation", p, hp);
  bool nest = true;
  for (const hl::Cluster& c : S.cl)
    for (int k = 0; k < 2; ++k)
      if (c.child[k] >= 0) {
        const hl::Cluster& ch = S.cl[c.child[k]];
        nest = nest && ch.lo >= c.lo && ch.hi <= c.hi && ch.lo < ch.hi;
      }
  check(nest, "clusters nest", p, hp);
  // leaves tile the index square: sum of areas and no overlap on a coarse check
  long long area = 0;
  bool inside = true;
  for (const hl::LeafInfo& l : S.lf) {
    area += (long long)l.m * l.n;
    inside = inside && l.rlo >= 0 && l.clo >= 0 && l.rlo + l.m <= N && l.clo + l.n <= N && l.m > 0 && l.n > 0;
  }
  check(inside, "leaves inside the matrix", p, hp);
  check(area == (long long)N * N, "leaves cover N^2 entries", p, hp);
  if (N <= 4096) {
    std::vector<unsigned char> cov((size_t)N * N, 0);
    bool once = true;
    for (const hl::LeafInfo& l : S.lf)
      for (int i = 0; i < l.m; ++i)
        for (int j = 0; j < l.n; ++j) once = once && ++cov[(size_t)(l.rlo + i) * N + (l.clo + j)] == 1;
    check(once, "every entry in exactly one leaf", p, hp);
  }
  const int P = (int)S.leafcl.size();
  bool lists = (int)S.rowptr.size() == P + 1 && (int)S.colptr.size() == P + 1;
  if (lists) {
    for (int q = 0; q < P && lists; ++q) {
      const hl::Cluster& c = S.cl[S.leafcl[q]];
      for (int e = S.rowptr[q]; e < S.rowptr[q + 1]; ++e) {
        const int li = S.rowidx[e];
        lists = lists && li >= 0 && li < (int)S.lf.size();
        if (lists) lists = S.lf[li].rlo <= c.lo && c.hi <= S.lf[li].rlo + S.lf[li].m;
      }
    }
  }
  check(lists, "row lists name the leaves over each leaf cluster", p, hp);
}

// masked domains, 2-means trees, variable order and Taylor blocks: the
// grid-index map holds exactly the kept points, in natural order through
// perm; every row's order index names its own value; no low-rank block is
// thinner than the Taylor rank
void masked_invariants(const hl::Structure& S, const std::vector<int32_t>& kept, const std::vector<double>& sf,
                       int taylor_rank, const hlevy_problem& p, const hlevy_hparams& hp) {
  bool lat_ok = S.lat.size() == (size_t)S.N && kept.size() == (size_t)S.N;
  for (int k = 0; lat_ok && k < S.N; ++k) lat_ok = S.lat[k] == kept[S.perm[k]];
  check(lat_ok, "grid index of every cluster position", p, hp);
  if (!sf.empty()) {
    bool var_ok = S.var_row.size() == (size_t)S.N;
    for (int k = 0; var_ok && k < S.N; ++k)
      var_ok = S.var_row[k] >= 0 && S.var_row[k] < (int)S.var_s.size() && S.var_s[S.var_row[k]] == sf[S.perm[k]];
    check(var_ok, "order index of every row", p, hp);
  }
  if (taylor_rank > 0) {
    bool thick = true;
    for (const hl::LeafInfo& l : S.lf) thick = thick && (l.kind != hl::K_LR || std::min(l.m, l.n) >= taylor_rank);
    check(thick, "no low-rank block thinner than the Taylor rank", p, hp);
  }
}

int masked_cases() {
  int built = 0;
  uint64_t state = 88172645463325252ull;   // xorshift64
  auto rnd = [&]() {
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return state;
  };
  for (int n : {16, 30, 31, 40, 61}) {
    for (int shape = 0; shape < 3; ++shape) {
      // 0: L-shape (the quadrant x >= 0, y >= 0 removed), 1: random 70 %, 2: a disc
      std::vector<uint8_t> mask((size_t)n * n);
      const double h = 2.0 / (n + 1);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          const double x = -1.0 + (i + 1) * h, y = -1.0 + (j + 1) * h;
          uint8_t m = 1;
          if (shape == 0) m = !(x >= 0.0 && y >= 0.0);
          if (shape == 1) m = (rnd() % 10) < 7;
          if (shape == 2) m = x * x + y * y < 0.8;
          mask[(size_t)i * n + j] = m;
        }
      std::vector<int32_t> kept;
      for (int g = 0; g < n * n; ++g)
        if (mask[g]) kept.push_back(g);
      std::vector<double> sf(kept.size());
      for (size_t k = 0; k < sf.size(); ++k) sf[k] = 0.1 + 0.8 * ((rnd() % 1000) / 1000.0) + 1e-4;
      for (int cluster : {HLEVY_CLUSTER_BISECT, HLEVY_CLUSTER_KMEANS})
        for (int leaf : {16, 32})
          for (int variant = 0; variant < 3; ++variant) {
            hlevy_problem p = problem(2, n);
            hlevy_hparams hp = hparams(leaf, 1.0, 4);
            hp.cluster = cluster;
            p.mask = mask.data();
            int tr = 0;
            if (variant == 1) {
              p.kernel = HLEVY_KERNEL_VARIABLE_ORDER;
              p.s_field = sf.data();
            } else if (variant == 2) {
              p.kernel = HLEVY_KERNEL_GAUSSIAN;
              p.eps2 = 5.0;
              hp.taylor_rank = tr = 10;
            }
            hl::Structure S;
            const std::string e = hl::build_structure(p, hp, S);
            if (!e.empty()) continue;   // e.g. fewer than two leaves
            ++built;
            invariants(S, p, hp);
            masked_invariants(S, kept, variant == 1 ? sf : std::vector<double>{}, tr, p, hp);
          }
    }
  }
  return built;
}

}  // namespace

int main() {
  int built = 0;
  for (int dim = 1; dim <= 2; ++dim) {
    const std::vector<int> ns = dim == 1 ? std::vector<int>{128, 129, 200, 1000, 1023, 4097, 65536}
                                         : std::vector<int>{12, 33, 40, 64, 100, 256};
    for (int n : ns)
      for (int leaf : {16, 32, 64})
        for (double eta : {0.5, 1.0, 2.0})
          for (int n_block : {1, 4, 64}) {
            hlevy_problem p = problem(dim, n);
            hlevy_hparams hp = hparams(leaf, eta, n_block);
            hl::Structure S;
            std::string e = hl::build_structure(p, hp, S);
            if (!e.empty()) continue;   // e.g. fewer than two leaves, or blocks above the row limit
            ++built;
            invariants(S, p, hp);
            // subdivide every third admissible block (seeded by position)
            std::set<std::pair<int32_t, int32_t>> sp;
            int k = 0;
            for (const hl::LeafInfo& l : S.lf)
              if (l.kind == hl::K_LR && (k++ % 3) == 0) sp.insert({l.r, l.c});
            if (!sp.empty() && S.N <= 4096) {
              hl::Structure S2;
              e = hl::build_structure(p, hp, S2, &sp);
              check(e.empty(), "subdivided structure builds", p, hp);
              if (e.empty()) invariants(S2, p, hp);
            }
          }
  }
  const int masked = masked_cases();
  built += masked;
  // invalid descriptors must be rejected, not crash
  int rejected = 0, bad = 0;
  std::vector<uint8_t> mask4(16, 1);
  std::vector<double> sbad(1024, 0.5);
  sbad[77] = 1.0;
  for (int variant = 0; variant < 16; ++variant) {
    hlevy_problem p = problem(1, 1024);
    hlevy_hparams hp = hparams(64, 1.0, 4);
    switch (variant) {
      case 0: p.dim = 3; break;
      case 1: p.n = 1; break;
      case 2: p.hi = p.lo; break;
      case 3: p.s = 1.0; break;
      case 4: p.a = -1.0; break;
      case 5: p.c = 1.0; break;
      case 6: p.r0 = 5.0; break;
      case 7: hp.leaf = 8; break;
      case 8: hp.max_rank = 99; break;
      case 9: p.n = 100; break;   // fewer than two leaves of 64
      case 10: p.kernel = 7; break;
      case 11: p.kernel = HLEVY_KERNEL_GAUSSIAN; p.eps2 = 0.0; hp.taylor_rank = 10; break;
      case 12: p.n = 4; p.mask = mask4.data(); break;                                // a mask in 1D
      case 13: hp.cluster = HLEVY_CLUSTER_KMEANS; break;                             // 2-means in 1D
      case 14: p.kernel = HLEVY_KERNEL_VARIABLE_ORDER; p.s_field = sbad.data(); break;  // s outside (0, 1)
      case 15: p.kernel = HLEVY_KERNEL_VARIABLE_ORDER; break;                        // no s_field
    }
    hl::Structure S;
    if (!hl::build_structure(p, hp, S).empty()) ++rejected; else ++bad;
  }
  if (bad) {
    ++failures;
    std::fprintf(stderr, "FAIL %d invalid descriptors accepted\n", bad);
  }
  std::printf("structures built %d (masked %d), invalid rejected %d, failures %d\n", built, masked, rejected,
              failures);
  return failures == 0 && built > 50 && masked > 50 ? 0 : 1;
}
