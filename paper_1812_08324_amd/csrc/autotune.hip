// Autotuner of the leaf size and the tile shapes of the per-step products
// (hlevy_autotune): every candidate is assembled, factored and stepped on
// the device through the public entry points, timed with the host clock
// around synchronised phases, and the fastest whole job per problem is kept
// in a JSON cache keyed by dimension, N bucket (nearest power of two),
// precision and batched-or-single.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "hl_internal.h"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// One cache entry.
struct TuneEntry {
  int leaf = 64, gather_waves = 0, rank_bucket = 0;
  double seconds = 0.0, default_seconds = 0.0;
};

// The cache file is the JSON object
//   {"version": 1, "entries": {"<key>": {"leaf": L, "gather_waves": W,
//    "rank_bucket": B, "seconds": S, "default_seconds": D}, ...}}
// written by save_cache; load_cache reads exactly that form (whitespace
// free) and ignores fields it does not know.
struct JsonReader {
  const std::string& s;
  size_t i = 0;
  bool ok = true;
  explicit JsonReader(const std::string& t) : s(t) {}
  void ws() {
    while (i < s.size() && (s[i] == ' ' || s[i] == '\n' || s[i] == '\r' || s[i] == '\t')) ++i;
  }
  bool eat(char c) {
    ws();
    if (i < s.size() && s[i] == c) {
      ++i;
      return true;
    }
    return false;
  }
  std::string str() {
    ws();
    std::string out;
    if (i >= s.size() || s[i] != '"') {
      ok = false;
      return out;
    }
    for (++i; i < s.size() && s[i] != '"'; ++i) out.push_back(s[i]);
    if (i >= s.size()) ok = false;
    ++i;
    return out;
  }
  double num() {
    ws();
    const char* b = s.c_str() + i;
    char* e = nullptr;
    const double v = std::strtod(b, &e);
    if (e == b) ok = false;
    i += (size_t)(e - b);
    return v;
  }
};

bool load_cache(const char* path, std::map<std::string, TuneEntry>& out) {
  std::ifstream f(path);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string text = ss.str();
  JsonReader r(text);
  if (!r.eat('{')) return false;
  while (r.ok && !r.eat('}')) {
    const std::string k = r.str();
    if (!r.eat(':')) return false;
    if (k == "entries") {
      if (!r.eat('{')) return false;
      while (r.ok && !r.eat('}')) {
        const std::string key = r.str();
        if (!r.eat(':') || !r.eat('{')) return false;
        TuneEntry e;
        while (r.ok && !r.eat('}')) {
          const std::string fld = r.str();
          if (!r.eat(':')) return false;
          const double v = r.num();
          if (fld == "leaf") e.leaf = (int)v;
          else if (fld == "gather_waves") e.gather_waves = (int)v;
          else if (fld == "rank_bucket") e.rank_bucket = (int)v;
          else if (fld == "seconds") e.seconds = v;
          else if (fld == "default_seconds") e.default_seconds = v;
          r.eat(',');
        }
        out[key] = e;
        r.eat(',');
      }
    } else {
      r.num();   // "version"
    }
    r.eat(',');
  }
  return r.ok;
}

bool save_cache(const char* path, const std::map<std::string, TuneEntry>& m) {
  std::ofstream f(path, std::ios::trunc);
  if (!f) return false;
  f << "{\n \"version\": 1,\n \"entries\": {";
  bool first = true;
  for (const auto& kv : m) {
    char buf[320];
    std::snprintf(buf, sizeof(buf),
                  "%s\n  \"%s\": {\"leaf\": %d, \"gather_waves\": %d, \"rank_bucket\": %d, \"seconds\": %.6e, "
                  "\"default_seconds\": %.6e}",
                  first ? "" : ",", kv.first.c_str(), kv.second.leaf, kv.second.gather_waves,
                  kv.second.rank_bucket, kv.second.seconds, kv.second.default_seconds);
    f << buf;
    first = false;
  }
  f << "\n }\n}\n";
  return (bool)f;
}

std::string tune_key(const hlevy_problem& p, int prec, bool batched) {
  const double N = p.dim == 1 ? (double)p.n : (double)p.n * p.n;
  char buf[96];
  std::snprintf(buf, sizeof(buf), "d%d_n%d_p%d_%s", p.dim, (int)std::lround(std::log2(N)), prec,
                batched ? "batched" : "single");
  return buf;
}

struct Handles {
  std::vector<hlevy_op*> ops;
  std::vector<hlevy_fac*> facs;
  std::vector<double*> us;
  ~Handles() {
    for (hlevy_fac* f : facs) hlevy_fac_destroy(f);
    for (hlevy_op* o : ops) hlevy_op_destroy(o);
    for (double* u : us) (void)hipFree(u);
  }
};

// Whole-job seconds per problem of one candidate: assembly and factorisation
// of `rep` copies (batched entry points when rep > 1), then nsteps steps at
// the rate of `timed` measured steps after two warm-up steps.  Returns a
// negative value when the candidate does not apply (the status says why).
double trial(const hlevy_problem& p, const hlevy_hparams& hp, double dt, int prec, double lu_tol, int64_t nsteps,
             int rep, hipStream_t s, hlevy_status& st) {
  Handles h;
  const int64_t N = p.dim == 1 ? (int64_t)p.n : (int64_t)p.n * p.n;
  const int timed = 20;
  if (hipStreamSynchronize(s) != hipSuccess) {
    st = HLEVY_ERR_DEVICE;
    return -1.0;
  }
  const double t0 = now_s();
  h.ops.assign(rep, nullptr);
  h.facs.assign(rep, nullptr);
  std::vector<hlevy_problem> ps(rep, p);
  std::vector<hlevy_hparams> hs(rep, hp);
  std::vector<double> dts(rep, dt);
  st = rep > 1 ? hlevy_assemble_batched(ps.data(), hs.data(), rep, nullptr, s, h.ops.data())
               : hlevy_assemble(&p, &hp, nullptr, s, h.ops.data());
  if (st != HLEVY_OK) {
    h.ops.clear();
    return -1.0;
  }
  st = rep > 1 ? hlevy_factor_batched(h.ops.data(), dts.data(), rep, prec, lu_tol, 0, s, h.facs.data())
               : hlevy_factor(h.ops[0], dt, prec, lu_tol, s, h.facs.data());
  if (st != HLEVY_OK) {
    h.facs.clear();
    return -1.0;
  }
  const double t1 = now_s();
  for (int r = 0; r < rep; ++r) {
    double* u = nullptr;
    if (hipMalloc(&u, (size_t)N * sizeof(double)) != hipSuccess) {
      st = HLEVY_ERR_OOM;
      return -1.0;
    }
    h.us.push_back(u);
    if (hipMemsetAsync(u, 0, (size_t)N * sizeof(double), s) != hipSuccess) {
      st = HLEVY_ERR_DEVICE;
      return -1.0;
    }
  }
  hlevy_refine rf{};
  rf.sweeps = 1;
  auto steps = [&](int k) -> hlevy_status {
    if (rep > 1) {
      std::vector<int64_t> ks(rep, k);
      return hlevy_step_batched(h.facs.data(), h.us.data(), ks.data(), rep, &rf, nullptr, s);
    }
    return hlevy_step(h.facs[0], h.us[0], k, nullptr, nullptr, &rf, nullptr, s);
  };
  if ((st = steps(2)) != HLEVY_OK) return -1.0;
  if (hipStreamSynchronize(s) != hipSuccess) {
    st = HLEVY_ERR_DEVICE;
    return -1.0;
  }
  const double t2 = now_s();
  if ((st = steps(timed)) != HLEVY_OK) return -1.0;
  if (hipStreamSynchronize(s) != hipSuccess) {
    st = HLEVY_ERR_DEVICE;
    return -1.0;
  }
  const double t3 = now_s();
  st = HLEVY_OK;
  return ((t1 - t0) + (double)nsteps * (t3 - t2) / timed) / rep;
}

}  // namespace

extern "C" {

hlevy_status hlevy_autotune(const hlevy_problem* prob, const hlevy_hparams* base, double dt, int32_t prec,
                            double lu_tol, int64_t nsteps, int32_t batch, const char* cache_path, void* stream,
                            hlevy_tune_result* out) {
  if (!prob || !base || !out) {
    hl::set_last_error("null argument");
    return HLEVY_ERR_INVALID_ARG;
  }
  if (prec != HLEVY_PREC_FP64 && prec != HLEVY_PREC_MIXED && prec != HLEVY_PREC_MIXED_BF16) {
    hl::set_last_error("bad precision");
    return HLEVY_ERR_INVALID_ARG;
  }
  if (!(dt > 0.0) || !std::isfinite(dt) || !(lu_tol > 0.0 && lu_tol < 1.0) || nsteps < 1 || batch < 1) {
    hl::set_last_error("need dt > 0, lu_tol in (0, 1), nsteps >= 1, batch >= 1");
    return HLEVY_ERR_INVALID_ARG;
  }
  {
    hl::Structure S;
    const std::string e = hl::build_structure(*prob, *base, S);
    if (!e.empty()) {
      hl::set_last_error(e);
      return HLEVY_ERR_INVALID_ARG;
    }
  }
  std::memset(out, 0, sizeof(*out));
  const std::string key = tune_key(*prob, prec, batch > 1);
  std::map<std::string, TuneEntry> cache;
  if (cache_path && *cache_path) load_cache(cache_path, cache);
  auto it = cache.find(key);
  if (it != cache.end()) {
    // cached: no device work at all
    out->leaf = it->second.leaf;
    out->gather_waves = it->second.gather_waves;
    out->rank_bucket = it->second.rank_bucket;
    out->seconds = it->second.seconds;
    out->default_seconds = it->second.default_seconds;
    out->from_cache = 1;
    return HLEVY_OK;
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int rep = batch > 1 ? std::min(batch, 8) : 1;
  // the caller's parameters first (the reference of default_seconds), then
  // leaf {64, 32} x gather width {auto, 4, 8} x rank bucket {auto, 16}
  std::vector<hlevy_hparams> cand;
  cand.push_back(*base);
  for (int leaf : {64, 32})
    for (int gw : {0, 4, 8})
      for (int kb : {0, 16}) {
        hlevy_hparams h = *base;
        h.leaf = leaf;
        h.gather_waves = gw;
        h.rank_bucket = kb;
        if (h.leaf == base->leaf && h.gather_waves == base->gather_waves && h.rank_bucket == base->rank_bucket)
          continue;
        cand.push_back(h);
      }
  // a warm-up trial (first launches of every kernel), not counted
  hlevy_status st = HLEVY_OK;
  if (trial(*prob, cand[0], dt, prec, lu_tol, nsteps, rep, s, st) < 0.0 && st != HLEVY_OK) return st;
  double best = -1.0;
  int ncand = 0;
  for (size_t c = 0; c < cand.size() && ncand < HLEVY_TUNE_MAX_CAND; ++c) {
    hl::Structure S;
    if (!hl::build_structure(*prob, cand[c], S).empty()) continue;   // e.g. N < 2 leaf
    const double t = trial(*prob, cand[c], dt, prec, lu_tol, nsteps, rep, s, st);
    if (t < 0.0) {
      if (c == 0) return st;
      continue;   // a shape the problem cannot take (reported through the count only)
    }
    out->cand_leaf[ncand] = cand[c].leaf;
    out->cand_gather_waves[ncand] = cand[c].gather_waves;
    out->cand_rank_bucket[ncand] = cand[c].rank_bucket;
    out->cand_seconds[ncand] = t;
    ++ncand;
    if (c == 0) out->default_seconds = t;
    if (best < 0.0 || t < best) {
      best = t;
      out->leaf = cand[c].leaf;
      out->gather_waves = cand[c].gather_waves;
      out->rank_bucket = cand[c].rank_bucket;
    }
  }
  out->ncand = ncand;
  out->seconds = best;
  out->from_cache = 0;
  if (cache_path && *cache_path) {
    TuneEntry e;
    e.leaf = out->leaf;
    e.gather_waves = out->gather_waves;
    e.rank_bucket = out->rank_bucket;
    e.seconds = out->seconds;
    e.default_seconds = out->default_seconds;
    cache[key] = e;
    if (!save_cache(cache_path, cache)) {
      hl::set_last_error(std::string("could not write the tuning cache ") + cache_path);
      return HLEVY_ERR_INVALID_ARG;
    }
  }
  return HLEVY_OK;
}

}  // extern "C"
