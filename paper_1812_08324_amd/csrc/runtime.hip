// Host runtime of the H-matrix Crank-Nicolson library: device storage of
// H-matrices, the batched plan of the H-LU with inverted triangular factors,
// its executor, and the C ABI declared in include/hlevy.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <deque>
#include <functional>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <chrono>
#include <cstdlib>
#include <vector>

#include "hl_internal.h"
#include "hl_jobs.h"
#include "hl_kernels.h"
#include "hl_mv.h"

namespace hl {

thread_local std::string g_last_error;

// Optional host-side phase timing on stderr (HLEVY_VERBOSE=1); level 2
// also prints the shape of every fused rounded-addition phase as planned.
static int verbose_level() {
  static int v = -1;
  if (v < 0) {
    const char* e = std::getenv("HLEVY_VERBOSE");
    v = (e && *e >= '1' && *e <= '9') ? *e - '0' : 0;
  }
  return v;
}
static bool verbose() { return verbose_level() >= 1; }
static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void set_last_error(const std::string& msg) { g_last_error = msg; }

static hlevy_status fail(hlevy_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HL_CHECK(expr)                                                                    \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      throw DeviceError(std::string(#expr) + ": " + hipGetErrorString(_e));               \
  } while (0)

struct DeviceError {
  std::string msg;
  explicit DeviceError(std::string m) : msg(std::move(m)) {}
};
struct OomError {
  std::string msg;
};

// ---------------------------------------------------------------------------
// device memory helpers
// ---------------------------------------------------------------------------
// Device memory goes through the caller's allocator when one was given to
// hlevy_assemble (the factor takes its operator's), else hipMalloc/hipFree.
// A buffer keeps the allocator and the byte counter of the handle that
// owns it from the scope active when it was allocated, so it is freed
// through the same allocator and uncounted from the same handle.
struct AllocCtx {
  hlevy_allocator al{};     // al.alloc == nullptr: hipMalloc / hipFree
  size_t* count = nullptr;  // resident bytes of the owning handle (nullptr: transient)
};
thread_local const AllocCtx* g_actx = nullptr;
struct AllocScope {
  const AllocCtx* prev;
  explicit AllocScope(const AllocCtx* c) : prev(g_actx) { g_actx = c; }
  ~AllocScope() { g_actx = prev; }
  AllocScope(const AllocScope&) = delete;
  AllocScope& operator=(const AllocScope&) = delete;
};
static void* dev_alloc(size_t b, const AllocCtx& c) {
  void* p = nullptr;
  if (c.al.alloc) {
    p = c.al.alloc(b, c.al.ctx);
    if (p && (reinterpret_cast<uintptr_t>(p) & 255)) {
      c.al.free(p, c.al.ctx);
      throw DeviceError("the caller's allocator returned memory not aligned to 256 bytes");
    }
  } else if (hipMalloc(&p, b) != hipSuccess) {
    (void)hipGetLastError();
    p = nullptr;
  }
  if (p && c.count) *c.count += b;
  return p;
}
static void dev_free(void* p, size_t b, const AllocCtx& c) {
  if (!p) return;
  if (c.al.alloc) c.al.free(p, c.al.ctx);
  else (void)hipFree(p);
  if (c.count) *c.count -= b;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  AllocCtx ctx{};
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { reset(); }
  void reset() {
    dev_free(p, bytes, ctx);
    p = nullptr;
    bytes = 0;
  }
  void alloc(size_t b) {
    reset();
    if (b == 0) b = 8;
    ctx = g_actx ? *g_actx : AllocCtx{};
    p = dev_alloc(b, ctx);
    if (!p) throw OomError{"device allocation of " + std::to_string(b) + " bytes failed"};
    bytes = b;
  }
  template <class T>
  T* as() const { return reinterpret_cast<T*>(p); }
};

template <class T>
static void upload(DevBuf& buf, const std::vector<T>& v, hipStream_t s) {
  buf.alloc(v.size() * sizeof(T));
  if (!v.empty()) HL_CHECK(hipMemcpyAsync(buf.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Stack allocator over device slabs: alloc/mark/release in LIFO order.
struct WsStack {
  struct Slab {
    char* p;
    size_t cap;
  };
  std::vector<Slab> slabs;
  size_t cur = 0, off = 0;
  size_t peak = 0, used_total = 0;
  AllocCtx ctx = g_actx ? *g_actx : AllocCtx{};
  static constexpr size_t SLAB = (size_t)256 << 20;
  ~WsStack() {
    for (auto& s : slabs) dev_free(s.p, s.cap, ctx);
  }
  struct Mark {
    size_t cur, off, used;
  };
  Mark mark() const { return {cur, off, used_total}; }
  void release(const Mark& m) {
    cur = m.cur;
    off = m.off;
    used_total = m.used;
  }
  double* alloc_d(size_t n) { return reinterpret_cast<double*>(alloc(n * sizeof(double))); }
  int32_t* alloc_i(size_t n) { return reinterpret_cast<int32_t*>(alloc(n * sizeof(int32_t))); }
  char* alloc(size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (;;) {
      if (cur < slabs.size() && off + bytes <= slabs[cur].cap) {
        char* p = slabs[cur].p + off;
        off += bytes;
        used_total += bytes;
        peak = std::max(peak, used_total);
        return p;
      }
      if (cur < slabs.size() && off > 0) {
        ++cur;
        off = 0;
        continue;
      }
      if (cur >= slabs.size() || slabs[cur].cap < bytes) {
        size_t cap = std::max(SLAB, bytes);
        void* p = dev_alloc(cap, ctx);
        if (!p) throw OomError{"workspace allocation of " + std::to_string(cap) + " bytes failed"};
        if (cur < slabs.size()) slabs.insert(slabs.begin() + cur, Slab{(char*)p, cap});
        else slabs.push_back(Slab{(char*)p, cap});
        off = 0;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// one H-matrix with the shared block structure
// ---------------------------------------------------------------------------
enum Shape { FULL = 0, LOWER = 1, UPPER = 2 };

// Bump allocator over one device buffer: the factorisation workspaces of a
// group of problems, reused from group to group without new allocations.
struct Arena {
  DevBuf buf;
  size_t off = 0;
  static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
  void reserve(size_t bytes) {
    if (buf.bytes < bytes) buf.alloc(bytes);
    off = 0;
  }
  char* take(size_t bytes) {
    bytes = round(std::max<size_t>(bytes, 8));
    if (off + bytes > buf.bytes) throw DeviceError("internal: factorisation arena overflow");
    char* p = reinterpret_cast<char*>(buf.p) + off;
    off += bytes;
    return p;
  }
};

struct HMat {
  const Structure* S = nullptr;
  std::vector<LeafDesc> L;
  DevBuf dL, drank, pool;     // owned storage (create); empty for arena storage (create_in)
  double* mem = nullptr;      // device leaf storage
  LeafDesc* ldev = nullptr;   // device copy of L
  int32_t* rank = nullptr;    // device, per leaf
  size_t pool_doubles = 0;
  std::vector<int32_t> pend;   // plan building: slot of the leaf's pending terms, or -1

  // dense_leaf_level: admissible blocks between two leaf clusters are held
  // dense in this matrix (the factorisation workspace), so that updates of
  // leaf-level blocks need no rounded addition.
  // leaf descriptors with offsets into the pool (no allocation); returns
  // the pool size in doubles
  size_t layout(const Structure& st, int kcap_max, Shape shape, bool dense_leaf_level) {
    S = &st;
    L.resize(st.lf.size());
    pend.assign(st.lf.size(), -1);
    size_t off = 0;
    for (size_t l = 0; l < st.lf.size(); ++l) {
      const LeafInfo& li = st.lf[l];
      LeafDesc d{};
      d.m = li.m;
      d.n = li.n;
      d.rlo = li.rlo;
      d.clo = li.clo;
      bool zero = (shape == LOWER && leaf_upper(li)) || (shape == UPPER && leaf_lower(li));
      d.kind = zero ? K_ZERO : li.kind;
      if (d.kind == K_LR && dense_leaf_level && st.leafpos[li.r] >= 0 && st.leafpos[li.c] >= 0) d.kind = K_DENSE;
      d.kcap = 0;
      if (d.kind == K_DENSE) {
        d.A = reinterpret_cast<double*>(off);
        off += ((size_t)li.m * li.n + 7) & ~(size_t)7;
      } else if (d.kind == K_LR) {
        d.kcap = std::min(kcap_max, std::min(li.m, li.n));
        d.A = reinterpret_cast<double*>(off);
        off += ((size_t)li.m * d.kcap + 7) & ~(size_t)7;
        d.B = reinterpret_cast<double*>(off);
        off += ((size_t)li.n * d.kcap + 7) & ~(size_t)7;
      }
      L[l] = d;
    }
    pool_doubles = off;
    return off;
  }
  void place(double* base) {
    mem = base;
    for (auto& d : L) {
      if (d.kind == K_DENSE) d.A = base + reinterpret_cast<size_t>(d.A);
      if (d.kind == K_LR) {
        d.A = base + reinterpret_cast<size_t>(d.A);
        d.B = base + reinterpret_cast<size_t>(d.B);
      }
    }
  }
  void create(const Structure& st, int kcap_max, Shape shape, hipStream_t s, bool dense_leaf_level = false) {
    layout(st, kcap_max, shape, dense_leaf_level);
    pool.alloc(std::max<size_t>(pool_doubles, 1) * sizeof(double));
    place(pool.as<double>());
    upload(dL, L, s);
    ldev = dL.as<LeafDesc>();
    drank.alloc(std::max<size_t>(L.size(), 1) * sizeof(int32_t));
    rank = drank.as<int32_t>();
    HL_CHECK(hipMemsetAsync(rank, 0, L.size() * sizeof(int32_t), s));
  }
  // storage taken from an arena (the arena outlives every use)
  static size_t arena_bytes(size_t pool_doubles, size_t nleaves) {
    return Arena::round(pool_doubles * sizeof(double)) + Arena::round(nleaves * sizeof(LeafDesc)) +
           Arena::round(nleaves * sizeof(int32_t)) + 3 * 256;
  }
  void create_in(Arena& a, const Structure& st, int kcap_max, Shape shape, hipStream_t s,
                 bool dense_leaf_level = false) {
    layout(st, kcap_max, shape, dense_leaf_level);
    place(reinterpret_cast<double*>(a.take(pool_doubles * sizeof(double))));
    ldev = reinterpret_cast<LeafDesc*>(a.take(L.size() * sizeof(LeafDesc)));
    if (!L.empty())
      HL_CHECK(hipMemcpyAsync(ldev, L.data(), L.size() * sizeof(LeafDesc), hipMemcpyHostToDevice, s));
    rank = reinterpret_cast<int32_t*>(a.take(L.size() * sizeof(int32_t)));
    HL_CHECK(hipMemsetAsync(rank, 0, L.size() * sizeof(int32_t), s));
  }
  const LeafDesc* dev() const { return ldev; }
};

// Device copies of the structure lists.
struct DevStructure {
  DevBuf rowptr, rowidx, colptr, colidx, lclo, lchi, perm, lat, ident;
  DevLists lists{};
  void create(const Structure& S, hipStream_t s) {
    upload(rowptr, S.rowptr, s);
    upload(rowidx, S.rowidx, s);
    upload(colptr, S.colptr, s);
    upload(colidx, S.colidx, s);
    std::vector<int32_t> lo, hi;
    for (int c : S.leafcl) {
      lo.push_back(S.cl[c].lo);
      hi.push_back(S.cl[c].hi);
    }
    upload(lclo, lo, s);
    upload(lchi, hi, s);
    upload(perm, S.perm, s);
    upload(lat, S.lat, s);
    std::vector<double> I(64 * 64, 0.0);
    for (int i = 0; i < 64; ++i) I[i + 64 * i] = 1.0;
    upload(ident, I, s);
    lists = DevLists{rowptr.as<int32_t>(), rowidx.as<int32_t>(), colptr.as<int32_t>(),
                     colidx.as<int32_t>(), lclo.as<int32_t>(), lchi.as<int32_t>()};
  }
};

// ---------------------------------------------------------------------------
// plan: phases over item arrays, built on the host, uploaded once
// ---------------------------------------------------------------------------
enum PhaseType {
  PH_APPLY, PH_DPROD, PH_DFLUSH, PH_LFLUSH, PH_COPY, PH_GETRF, PH_LUINV, PH_RADD,
  // deferred work: the phases between DEFER_BEGIN and DEFER_END run on the
  // deferred stream (after all earlier phases of the caller's stream); the
  // caller's stream waits for them at DEFER_JOIN (strictly nested pairs)
  PH_DEFER_BEGIN, PH_DEFER_END, PH_DEFER_JOIN
};

struct Phase {
  int type;
  int b0, n0, b1, n1, b2, n2;
  double tol;
  int ks;        // PH_LFLUSH: LDS stride, >= the widest concatenation of the phase
  // side > 0: this phase and the next side - 1 run on the side stream, and
  // the par phases after them (on the caller's stream) touch none of their
  // data; the streams join after those
  int side = 0, par = 0;
};

// A second stream (default priority) and two events per device and host
// thread, kept for the life of the thread: a fused rounded-addition launch
// runs there while the independent phases after it run on the caller's
// stream (one set per thread, so concurrent callers never share events).
struct ForkJoin {
  hipStream_t side = nullptr, deferred = nullptr;
  hipEvent_t fork = nullptr, join = nullptr, dfork = nullptr, djoin = nullptr;
  // plan segments are copied to the device on their own stream: a copy from
  // pageable memory waits for its stream to drain, which on the caller's
  // stream would hold the host until every earlier segment had run
  hipStream_t upload = nullptr;
  hipEvent_t uploaded = nullptr;
};
static ForkJoin& fork_join() {
  static thread_local std::map<int, ForkJoin> per_device;
  int dev = 0;
  HL_CHECK(hipGetDevice(&dev));
  ForkJoin& f = per_device[dev];
  if (!f.side) {
    HL_CHECK(hipStreamCreateWithFlags(&f.side, hipStreamNonBlocking));
    HL_CHECK(hipStreamCreateWithFlags(&f.deferred, hipStreamNonBlocking));
    HL_CHECK(hipEventCreateWithFlags(&f.fork, hipEventDisableTiming));
    HL_CHECK(hipEventCreateWithFlags(&f.join, hipEventDisableTiming));
    HL_CHECK(hipEventCreateWithFlags(&f.dfork, hipEventDisableTiming));
    HL_CHECK(hipEventCreateWithFlags(&f.djoin, hipEventDisableTiming));
    HL_CHECK(hipStreamCreateWithFlags(&f.upload, hipStreamNonBlocking));
    HL_CHECK(hipEventCreateWithFlags(&f.uploaded, hipEventDisableTiming));
  }
  return f;
}

struct Plan {
  std::vector<Phase> ph;
  std::vector<ApplyJob> jobs;
  std::vector<ProjItem> proj;
  std::vector<GatherItem> gath;
  std::vector<DProdItem> dprod;
  std::vector<Term> terms;
  std::vector<DFlushItem> dflush;
  std::vector<LFlushTarget> ltg;
  std::vector<ChunkItem> lgram, lexp;
  std::vector<CopyItem> copies;
  std::vector<GetrfItem> getrf;
  std::vector<LuInvItem> luinv;
  DevBuf djobs, dproj, dgath, ddprod, dterms, ddflush, dltg, dlgram, dlexp, dcopies, dgetrf, dluinv;

  // Exchanges the whole plan (host arrays and device copies) with o.
  void swap_contents(Plan& o) {
    ph.swap(o.ph);
    jobs.swap(o.jobs);
    proj.swap(o.proj);
    gath.swap(o.gath);
    dprod.swap(o.dprod);
    terms.swap(o.terms);
    dflush.swap(o.dflush);
    ltg.swap(o.ltg);
    lgram.swap(o.lgram);
    lexp.swap(o.lexp);
    copies.swap(o.copies);
    getrf.swap(o.getrf);
    luinv.swap(o.luinv);
    for (auto pr : {std::make_pair(&djobs, &o.djobs), std::make_pair(&dproj, &o.dproj),
                    std::make_pair(&dgath, &o.dgath), std::make_pair(&ddprod, &o.ddprod),
                    std::make_pair(&dterms, &o.dterms), std::make_pair(&ddflush, &o.ddflush),
                    std::make_pair(&dltg, &o.dltg), std::make_pair(&dlgram, &o.dlgram),
                    std::make_pair(&dlexp, &o.dlexp), std::make_pair(&dcopies, &o.dcopies),
                    std::make_pair(&dgetrf, &o.dgetrf), std::make_pair(&dluinv, &o.dluinv)}) {
      std::swap(pr.first->p, pr.second->p);
      std::swap(pr.first->bytes, pr.second->bytes);
      std::swap(pr.first->ctx, pr.second->ctx);
    }
  }

  // Host-side check of the plan before it reaches the device: every phase's
  // item range lies inside its array, every term of a rounded addition or
  // dense flush has at least one row and one column inside its target and
  // non-null factors.  Violations are planner bugs: they become an error
  // instead of an out-of-bounds access on the device.
  void validate() const {
    auto bad = [](const std::string& what) { throw DeviceError("internal: plan check failed: " + what); };
    auto in_range = [&](int b, int n, size_t size, const char* what) {
      if (b < 0 || n < 0 || (size_t)b + (size_t)n > size) bad(std::string(what) + " item range");
    };
    auto check_terms = [&](int tbeg, int tcount, int m, int n) {
      in_range(tbeg, tcount, terms.size(), "term");
      for (int t = tbeg; t < tbeg + tcount; ++t) {
        const Term& tm = terms[t];
        if (tm.mr < 1 || tm.nc < 1 || tm.ro < 0 || tm.co < 0 || tm.ro + tm.mr > m || tm.co + tm.nc > n)
          bad("term outside its target");
        if (!tm.U || (tm.dense != 1 && !tm.W)) bad("null term factor");
        if (tm.dense == 2 && tm.kfix < 1) bad("product term without inner dimension");
        if (tm.dense == 0 && !tm.k && tm.kfix < 0) bad("negative term rank");
      }
    };
    for (const LFlushTarget& T : ltg) {
      if (T.m < 1 || T.n < 1 || !T.U || !T.V || T.kcap < 0 || T.Kcap > KMAX || !T.info) bad("low-rank target");
      check_terms(T.tbeg, T.tcount, T.m, T.n);
    }
    for (const DFlushItem& D : dflush) {
      if (D.m < 1 || D.n < 1 || D.m > 64 || D.n > 64 || !D.D) bad("dense target");
      check_terms(D.tbeg, D.tcount, D.m, D.n);
    }
    for (const ChunkItem& c : lgram)
      if (c.tgt < 0 || c.r0 < 0 || c.r1 <= c.r0) bad("Gram chunk");
    for (const ChunkItem& c : lexp)
      if (c.tgt < 0 || c.r0 < 0 || c.r1 <= c.r0) bad("expand chunk");
    for (const Phase& p : ph) {
      switch (p.type) {
        case PH_APPLY: in_range(p.b0, p.n0, proj.size(), "projection"); in_range(p.b1, p.n1, gath.size(), "gather"); break;
        case PH_DPROD: in_range(p.b0, p.n0, dprod.size(), "product"); break;
        case PH_DFLUSH: in_range(p.b0, p.n0, dflush.size(), "dense flush"); break;
        case PH_LFLUSH:
          in_range(p.b0, p.n0, ltg.size(), "low-rank target");
          in_range(p.b1, p.n1, lgram.size(), "Gram chunk");
          in_range(p.b2, p.n2, lexp.size(), "expand chunk");
          // the chunked kernels take a target's whole term list as one
          // concatenation (at most 64 terms); the fused kernel takes any
          // number of terms in concatenations of its own
          for (int q = p.b0; q < p.b0 + p.n0; ++q)
            if (ltg[q].tcount > 64) bad("more than 64 terms in one chunked rounded addition");
          for (int q = p.b1; q < p.b1 + p.n1; ++q)
            if (lgram[q].tgt >= p.n0) bad("Gram chunk target");
          for (int q = p.b2; q < p.b2 + p.n2; ++q)
            if (lexp[q].tgt >= p.n0) bad("expand chunk target");
          break;
        case PH_RADD: in_range(p.b0, p.n0, ltg.size(), "fused target"); in_range(p.b1, p.n1, dflush.size(), "dense flush"); break;
        case PH_COPY: in_range(p.b0, p.n0, copies.size(), "copy"); break;
        case PH_GETRF: in_range(p.b0, p.n0, getrf.size(), "leaf factorisation"); break;
        case PH_LUINV: in_range(p.b0, p.n0, luinv.size(), "diagonal node"); break;
        default: break;
      }
    }
  }

  void upload_all(hipStream_t s) {
    validate();
    upload(djobs, jobs, s);
    upload(dproj, proj, s);
    upload(dgath, gath, s);
    upload(ddprod, dprod, s);
    upload(dterms, terms, s);
    upload(ddflush, dflush, s);
    upload(dltg, ltg, s);
    upload(dlgram, lgram, s);
    upload(dlexp, lexp, s);
    upload(dcopies, copies, s);
    upload(dgetrf, getrf, s);
    upload(dluinv, luinv, s);
  }

  void run(int32_t* zero_pivot, hipStream_t s) const {
    // a PH_RADD phase with par > 0 goes to the side stream; the join waits
    // after the par phases that follow it
    size_t join_at = (size_t)-1;
    ForkJoin* fj = nullptr;
    bool in_deferred = false;
    for (size_t q = 0; q < ph.size(); ++q) {
      if (q == join_at) {
        HL_CHECK(hipEventRecord(fj->join, fj->side));
        HL_CHECK(hipStreamWaitEvent(s, fj->join, 0));
        join_at = (size_t)-1;
      }
      const Phase& p = ph[q];
      if (p.type == PH_DEFER_BEGIN) {
        fj = &fork_join();
        HL_CHECK(hipEventRecord(fj->dfork, s));
        HL_CHECK(hipStreamWaitEvent(fj->deferred, fj->dfork, 0));
        in_deferred = true;
        continue;
      }
      if (p.type == PH_DEFER_END) {
        in_deferred = false;
        continue;
      }
      if (p.type == PH_DEFER_JOIN) {
        fj = &fork_join();
        HL_CHECK(hipEventRecord(fj->djoin, fj->deferred));
        HL_CHECK(hipStreamWaitEvent(s, fj->djoin, 0));
        continue;
      }
      if (in_deferred) {   // in order on the deferred stream, no side forks
        run_phase(p, zero_pivot, fork_join().deferred);
        continue;
      }
      if (p.side > 0 && p.par > 0 && join_at == (size_t)-1) {
        fj = &fork_join();
        HL_CHECK(hipEventRecord(fj->fork, s));
        HL_CHECK(hipStreamWaitEvent(fj->side, fj->fork, 0));
        for (int u = 0; u < p.side; ++u) run_phase(ph[q + u], zero_pivot, fj->side);
        join_at = q + (size_t)p.side + (size_t)p.par;
        q += (size_t)p.side - 1;
        continue;
      }
      run_phase(p, zero_pivot, s);
    }
    if (join_at != (size_t)-1) {
      HL_CHECK(hipEventRecord(fj->join, fj->side));
      HL_CHECK(hipStreamWaitEvent(s, fj->join, 0));
    }
    if (in_deferred) throw DeviceError("internal: deferred phases without an end");
  }

  void run_phase(const Phase& p, int32_t* zero_pivot, hipStream_t s) const {
    {
      switch (p.type) {
        case PH_APPLY:
          HL_CHECK(launch_apply(djobs.as<ApplyJob>(), dproj.as<ProjItem>() + p.b0, p.n0,
                                dgath.as<GatherItem>() + p.b1, p.n1, s));
          break;
        case PH_DPROD:
          HL_CHECK(launch_dense_prod(ddprod.as<DProdItem>() + p.b0, p.n0, s));
          break;
        case PH_DFLUSH:
          HL_CHECK(launch_flush_dense(ddflush.as<DFlushItem>() + p.b0, p.n0, dterms.as<Term>(), s));
          break;
        case PH_LFLUSH:
          HL_CHECK(launch_flush_lr(dltg.as<LFlushTarget>() + p.b0, p.n0, dterms.as<Term>(),
                                   dlgram.as<ChunkItem>() + p.b1, p.n1, dlexp.as<ChunkItem>() + p.b2,
                                   p.n2, p.tol, p.ks, s));
          break;
        case PH_COPY:
          HL_CHECK(launch_copy(dcopies.as<CopyItem>() + p.b0, p.n0, s));
          break;
        case PH_GETRF:
          HL_CHECK(launch_getrf_inv(dgetrf.as<GetrfItem>() + p.b0, p.n0, zero_pivot, s));
          break;
        case PH_RADD:
          // b1, n1: dense flushes of the same batch that share the launch
          HL_CHECK(launch_radd_fused(dltg.as<LFlushTarget>() + p.b0, p.n0, dterms.as<Term>(), p.tol, p.ks, s,
                                     ddflush.as<DFlushItem>() + p.b1, p.n1, dterms.as<Term>()));
          break;
        case PH_LUINV:
          HL_CHECK(launch_lu_inv(dluinv.as<LuInvItem>() + p.b0, p.n0, zero_pivot, s));
          break;
      }
    }
  }
};

// Chunk items for a rounded addition of target index `t` in the plan.
static void add_chunks(Plan& P, int t, int m, int n, LFlushTarget& T, int gram_base_unused) {
  (void)gram_base_unused;
  T.nchA = (m + GRAM_CHUNK - 1) / GRAM_CHUNK;
  T.nchB = (n + GRAM_CHUNK - 1) / GRAM_CHUNK;
  for (int side = 0; side < 2; ++side) {
    int len = side == 0 ? m : n;
    int nch = side == 0 ? T.nchA : T.nchB;
    for (int c = 0; c < nch; ++c) {
      ChunkItem ci{t, side, c * GRAM_CHUNK, std::min(len, (c + 1) * GRAM_CHUNK), c, 0};
      P.lgram.push_back(ci);
      P.lexp.push_back(ci);
    }
  }
}

static size_t flush_ws_doubles(const LFlushTarget& T) {
  return (size_t)(T.nchA + T.nchB) * npairs_host(T.Kcap) * 2 + (size_t)2 * T.Kcap * 32;
}

// ---------------------------------------------------------------------------
// builder of the factorisation plan
// ---------------------------------------------------------------------------
struct PendingTerm {
  Term t;
  int kcap;   // capacity bound of the term's rank
};

// The builder takes work of several problems at once: every matrix carries its
// own block structure, and the products, copies and rounded additions of one
// batch land in the same phases whichever problem they belong to.
struct Builder {
  Plan& P;
  WsStack& ws;
  const double* ident;   // 64 x 64 identity on the device
  int32_t* overflow;
  double tol;
  std::map<const Structure*, DevLists> lists_of;
  // batch state
  std::vector<ApplyJob> bjobs;
  std::vector<const HMat*> bjob_mat;
  std::vector<DProdItem> bdprod;
  // pending update terms per target leaf, in slots (HMat::pend indexes them)
  std::vector<std::pair<HMat*, int>> pkeys;
  std::vector<std::vector<PendingTerm>> pterms;
  struct PendView {
    std::pair<HMat*, int> first;
    std::vector<PendingTerm>& second;
  };
  WsStack::Mark mk{};
  bool in_batch = false;
  // inside a PH_DEFER_BEGIN .. PH_DEFER_END region
  bool in_defer = false;
  // called after every batch outside a deferred region: the point where the
  // plan built so far may be handed to the device (nothing built later
  // refers to its items by index)
  std::function<void()> after_batch;

  Builder(Plan& p, WsStack& w, const double* id, int32_t* ovf, double t)
      : P(p), ws(w), ident(id), overflow(ovf), tol(t) {}

  // registers the block structure of a problem (its leaf-cluster lists)
  void add_problem(const Structure& S, const DevStructure& ds) { lists_of[&S] = ds.lists; }

  void begin() {
    mk = ws.mark();
    in_batch = true;
  }

  void add_apply(HMat* M, int node, int trans, const double* X, int ldx, const int32_t* kx, int kxcap,
                 double* Y, int ldy) {
    const Structure& S = *M->S;
    const BNode& b = S.bn[node];
    ApplyJob J{};
    auto li = lists_of.find(&S);
    if (li == lists_of.end()) throw DeviceError("internal: unregistered block structure");
    J.dl = li->second;
    J.L = M->dev();
    J.rank = M->rank;
    J.lbeg = b.lbeg;
    J.lend = b.lend;
    J.rlo = S.cl[b.r].lo;
    J.rhi = S.cl[b.r].hi;
    J.clo = S.cl[b.c].lo;
    J.chi = S.cl[b.c].hi;
    J.trans = trans;
    J.ldx = ldx;
    J.ldy = ldy;
    J.kxcap = kxcap;
    J.X = X;
    J.kx = kx;
    J.Y = Y;
    J.tstride = 32 * kxcap;
    J.T = ws.alloc_d((size_t)(b.lend - b.lbeg) * J.tstride);
    bjobs.push_back(J);
    bjob_mat.push_back(M);
  }

  // push a term covering rows [r0, r1) x cols [c0, c1) (absolute) into the
  // target node of matrix C
  void push(HMat* C, int cnode, Term t, int kcap, int r0, int r1, int c0, int c1) {
    const Structure& S = *C->S;
    const BNode& c = S.bn[cnode];
    if (c.kind == K_H) {
      for (int q = 0; q < 4; ++q) {
        const BNode& ch = S.bn[c.child[q]];
        int a0 = std::max(r0, S.cl[ch.r].lo), a1 = std::min(r1, S.cl[ch.r].hi);
        int b0 = std::max(c0, S.cl[ch.c].lo), b1 = std::min(c1, S.cl[ch.c].hi);
        if (a0 >= a1 || b0 >= b1) continue;
        Term u = t;
        if (t.dense == 1) {
          u.U = t.U + (a0 - r0) + (size_t)t.ldu * (b0 - c0);
        } else if (t.dense == 2) {
          u.U = t.U + (a0 - r0);                       // rows of the left factor
          u.W = t.W + (size_t)t.ldw * (b0 - c0);       // columns of the right factor
        } else {
          u.U = t.U + (a0 - r0);
          u.W = t.W + (b0 - c0);
        }
        push(C, c.child[q], u, kcap, a0, a1, b0, b1);
      }
      return;
    }
    const LeafDesc& d = C->L[c.leaf];
    if (d.kind == K_ZERO) throw DeviceError("internal: update of a structurally zero block");
    t.ro = r0 - d.rlo;
    t.mr = r1 - r0;
    t.co = c0 - d.clo;
    t.nc = c1 - c0;
    int32_t& slot = C->pend[c.leaf];
    if (slot < 0) {
      slot = (int32_t)pkeys.size();
      pkeys.push_back({C, c.leaf});
      pterms.emplace_back();
    }
    pterms[slot].push_back({t, kcap});
  }

  // C[cnode region] += sign * A[an] * B[bn]
  void mma(HMat* C, int cnode, HMat* A, int an, HMat* B, int bnd, double sign) {
    const Structure& S = *C->S;
    if (A->S != C->S || B->S != C->S) throw DeviceError("internal: product across problems");
    const BNode& a = S.bn[an];
    const BNode& b = S.bn[bnd];
    int ak = a.kind == K_H ? (int)K_H : A->L[a.leaf].kind;
    int bk = b.kind == K_H ? (int)K_H : B->L[b.leaf].kind;
    if (ak == K_ZERO || bk == K_ZERO) return;
    const int r0 = S.cl[a.r].lo, r1 = S.cl[a.r].hi, c0 = S.cl[b.c].lo, c1 = S.cl[b.c].hi;
    if (ak == K_LR) {
      const LeafDesc& la = A->L[a.leaf];
      int nrow = c1 - c0;
      double* W = ws.alloc_d((size_t)nrow * la.kcap);
      add_apply(B, bnd, 1, la.B, la.n, A->rank + a.leaf, la.kcap, W, nrow);
      Term t{};
      t.dense = 0;
      t.U = la.A;
      t.ldu = la.m;
      t.W = W;
      t.ldw = nrow;
      t.k = A->rank + a.leaf;
      t.sign = sign;
      push(C, cnode, t, la.kcap, r0, r1, c0, c1);
    } else if (bk == K_LR) {
      const LeafDesc& lb = B->L[b.leaf];
      int nrow = r1 - r0;
      double* Z = ws.alloc_d((size_t)nrow * lb.kcap);
      add_apply(A, an, 0, lb.A, lb.m, B->rank + b.leaf, lb.kcap, Z, nrow);
      Term t{};
      t.dense = 0;
      t.U = Z;
      t.ldu = nrow;
      t.W = lb.B;
      t.ldw = lb.n;
      t.k = B->rank + b.leaf;
      t.sign = sign;
      push(C, cnode, t, lb.kcap, r0, r1, c0, c1);
    } else if (ak == K_DENSE && bk == K_DENSE) {
      // a product term: dense targets take it as it is, low-rank targets
      // get the product formed first (end())
      const LeafDesc& la = A->L[a.leaf];
      const LeafDesc& lb = B->L[b.leaf];
      Term t{};
      t.dense = 2;
      t.U = la.A;
      t.ldu = la.m;
      t.W = lb.A;
      t.ldw = lb.m;
      t.kfix = la.n;
      t.sign = sign;
      push(C, cnode, t, std::min(32, std::min(la.m, lb.n)), r0, r1, c0, c1);
    } else {
      if (!(ak == K_H && bk == K_H)) throw DeviceError("internal: inconsistent block tree levels");
      const BNode& c = S.bn[cnode];
      for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) {
          int cc = c.kind == K_H ? c.child[2 * i + j] : cnode;
          for (int k = 0; k < 2; ++k) mma(C, cc, A, a.child[2 * i + k], B, b.child[2 * k + j], sign);
        }
    }
  }

  // Emit rounded additions for the given targets.  Targets of at most
  // GRAM_CHUNK rows on both sides and at most fused_width(ftol) columns in
  // all (48, or 64 without double-double parts) go to one fused launch; the
  // others get one phase per width bucket (16, 32, 48, 64 columns) so that
  // the LDS of the core kernel is sized to the bucket.
  // Returns each target's index in P.ltg.
  std::vector<int> emit_lflush(std::vector<LFlushTarget>& tgs, std::vector<std::vector<Term>>& tlists,
                               double ftol) {
    std::vector<int> where(tgs.size(), -1);
    std::vector<size_t> fused;
    int fks = 16;
    for (size_t q = 0; q < tgs.size(); ++q)
      if (tgs[q].m <= GRAM_CHUNK && tgs[q].n <= GRAM_CHUNK && tgs[q].Kcap <= fused_width(ftol)) {
        fused.push_back(q);
        fks = std::max(fks, (tgs[q].Kcap + 15) / 16 * 16);
      }
    if (!fused.empty() && verbose_level() >= 2) {
      int tmax = 0, tsum = 0, mmax = 0;
      for (size_t q : fused) {
        tmax = std::max(tmax, (int)tlists[q].size());
        tsum += (int)tlists[q].size();
        mmax = std::max(mmax, std::max(tgs[q].m, tgs[q].n));
      }
      std::fprintf(stderr, "[hlevy] radd phase: targets %zu terms max %d mean %.1f rows<= %d\n", fused.size(),
                   tmax, (double)tsum / fused.size(), mmax);
    }
    if (!fused.empty()) {
      Phase ph{PH_RADD, (int)P.ltg.size(), (int)fused.size(), 0, 0, 0, 0, ftol, fks};
      for (size_t q : fused) {
        LFlushTarget T = tgs[q];
        T.tbeg = (int)P.terms.size();
        T.tcount = (int)tlists[q].size();
        for (auto& tm : tlists[q]) P.terms.push_back(tm);
        T.nchA = T.nchB = 1;
        T.ws = nullptr;
        T.info = ws.alloc_i(4);
        T.overflow = overflow;
        where[q] = (int)P.ltg.size();
        P.ltg.push_back(T);
      }
      P.ph.push_back(ph);
    }
    for (int bucket = 16; bucket <= KMAX; bucket += 16) {
      std::vector<size_t> sel;
      for (size_t q = 0; q < tgs.size(); ++q)
        if (where[q] < 0 && tgs[q].Kcap <= bucket && tgs[q].Kcap > bucket - 16) sel.push_back(q);
      if (sel.empty()) continue;
      Phase ph{PH_LFLUSH, (int)P.ltg.size(), (int)sel.size(), (int)P.lgram.size(), 0, (int)P.lexp.size(), 0,
               ftol, bucket};
      for (size_t q : sel) {
        LFlushTarget T = tgs[q];
        T.tbeg = (int)P.terms.size();
        T.tcount = (int)tlists[q].size();
        if (T.tcount > 64) throw DeviceError("internal: more than 64 terms in one rounded addition");
        for (auto& tm : tlists[q]) P.terms.push_back(tm);
        int tix = (int)P.ltg.size();
        add_chunks(P, tix - ph.b0, T.m, T.n, T, 0);
        T.ws = ws.alloc_d(flush_ws_doubles(T));
        T.info = ws.alloc_i(4);
        T.overflow = overflow;
        where[q] = tix;
        P.ltg.push_back(T);
      }
      ph.n1 = (int)P.lgram.size() - ph.b1;
      ph.n2 = (int)P.lexp.size() - ph.b2;
      P.ph.push_back(ph);
    }
    return where;
  }

  // A low-rank target whose rounded additions all run in one fused launch:
  // at most GRAM_CHUNK rows per side and rank capacities such that each
  // concatenation of the fused kernel (the target and one more term at
  // least) stays within fused_width(tol): target <= 16 and terms <= 32 with
  // double-double parts, both <= 32 without (called after the dense terms
  // became low-rank terms).
  bool fused_target(const LeafDesc& d, const std::vector<PendingTerm>& terms) const {
    const int tcap = radd_dd(tol) ? 16 : 32;
    if (d.kind != K_LR || d.m > GRAM_CHUNK || d.n > GRAM_CHUNK || d.kcap > tcap) return false;
    for (const auto& pt : terms)
      if (pt.t.dense || pt.kcap > 32) return false;
    return true;
  }

  // keep_ws: leave the batch's workspace allocated (its phases run on the
  // deferred stream and may still be running when later batches start); the
  // caller releases it with release_kept(mark) once the stream has joined.
  WsStack::Mark end(bool keep_ws = false) {
    // 1. applies (all independent within the batch)
    const size_t ph_apply = bjobs.empty() ? (size_t)-1 : P.ph.size();
    if (!bjobs.empty()) {
      int jb = (int)P.jobs.size();
      Phase ph{PH_APPLY, (int)P.proj.size(), 0, (int)P.gath.size(), 0, 0, 0, 0.0};
      for (size_t q = 0; q < bjobs.size(); ++q) {
        const ApplyJob& J = bjobs[q];
        const Structure& S = *bjob_mat[q]->S;
        P.jobs.push_back(J);
        for (int l = J.lbeg; l < J.lend; ++l)
          if (bjob_mat[q]->L[l].kind == K_LR) P.proj.push_back(ProjItem{jb + (int)q, l});
        // leaf clusters inside [o0, o1): a contiguous run of leafcl (index order)
        const int o0 = J.trans ? J.clo : J.rlo, o1 = J.trans ? J.chi : J.rhi;
        size_t lp = std::partition_point(S.leafcl.begin(), S.leafcl.end(),
                                         [&](int32_t c) { return S.cl[c].lo < o0; }) - S.leafcl.begin();
        for (; lp < S.leafcl.size() && S.cl[S.leafcl[lp]].hi <= o1; ++lp)
          P.gath.push_back(GatherItem{jb + (int)q, (int)lp});
      }
      ph.n0 = (int)P.proj.size() - ph.b0;
      ph.n1 = (int)P.gath.size() - ph.b1;
      P.ph.push_back(ph);
    }
    // targets in (matrix, leaf) order
    std::vector<PendView> pending;
    {
      std::vector<int> ord(pkeys.size());
      for (size_t q = 0; q < ord.size(); ++q) ord[q] = (int)q;
      std::sort(ord.begin(), ord.end(), [&](int a, int b) { return pkeys[a] < pkeys[b]; });
      pending.reserve(ord.size());
      for (int q : ord) pending.push_back(PendView{pkeys[q], pterms[q]});
    }
    // 2. products into low-rank targets are formed densely (workspace),
    //    then compressed below; dense targets take product terms as they are
    for (auto& kv : pending) {
      HMat* C = kv.first.first;
      if (C->L[kv.first.second].kind != K_LR) continue;
      for (auto& pt : kv.second) {
        if (pt.t.dense != 2) continue;
        Term& t = pt.t;
        double* Pp = ws.alloc_d((size_t)t.mr * t.nc);
        bdprod.push_back(DProdItem{t.U, t.W, Pp, t.ldu, t.ldw, t.mr, t.mr, t.kfix, t.nc});
        t.dense = 1;
        t.U = Pp;
        t.ldu = t.mr;
        t.W = nullptr;
      }
    }
    const size_t ph_dprod = bdprod.empty() ? (size_t)-1 : P.ph.size();
    if (!bdprod.empty()) {
      Phase ph{PH_DPROD, (int)P.dprod.size(), (int)bdprod.size(), 0, 0, 0, 0, 0.0};
      for (auto& d : bdprod) P.dprod.push_back(d);
      P.ph.push_back(ph);
    }
    // 3. dense terms into low-rank targets are compressed on their own
    //    first, 32 columns at a time (P = [P1 P2] = P1 I1^T + P2 I2^T), so
    //    that every rounded addition stays within 48 columns
    {
      struct Comp {
        LFlushTarget T;
        Term src;     // the dense term
        int kc;
      };
      std::vector<Comp> comps;
      for (auto& kv : pending) {
        HMat* C = kv.first.first;
        const LeafDesc& d = C->L[kv.first.second];
        if (d.kind != K_LR) continue;
        for (auto& pt : kv.second) {
          if (!pt.t.dense) continue;
          const int mr = pt.t.mr, nc = pt.t.nc;
          const int kc = std::min(std::min(d.kcap, 32), std::min(mr, nc));
          Comp c{};
          c.T.U = ws.alloc_d((size_t)mr * kc);
          c.T.V = ws.alloc_d((size_t)nc * kc);
          c.T.rank = ws.alloc_i(1);
          c.T.m = mr;
          c.T.n = nc;
          c.T.kcap = kc;
          c.src = pt.t;
          c.kc = kc;
          comps.push_back(c);
        }
      }
      if (!comps.empty()) {
        // every temporary in one fused launch: it starts empty (rank pointer
        // null, the kernel keeps the rank and leaves it in info[1]) and takes
        // the dense block as terms P[:, c0:c1] I^T of w columns, kc + w <= 48
        std::vector<LFlushTarget> tgs;
        std::vector<std::vector<Term>> tl;
        for (auto& c : comps) {
          LFlushTarget T = c.T;
          T.rank = nullptr;
          // one concatenation takes the whole block when the fused kernel
          // is 64 columns wide (no double-double parts)
          T.Kcap = fused_width(tol);
          T.borth = 1;
          const int w = c.kc <= 16 ? 32 : 16;
          std::vector<Term> terms;
          for (int c0 = 0; c0 < c.src.nc; c0 += w) {
            const int c1 = std::min(c.src.nc, c0 + w);
            Term lt{};
            lt.dense = 0;
            lt.ro = 0;
            lt.mr = c.src.mr;
            lt.co = c0;
            lt.nc = c1 - c0;
            lt.U = c.src.U + (size_t)c.src.ldu * c0;
            lt.ldu = c.src.ldu;
            lt.W = ident;
            lt.ldw = 64;
            lt.kfix = c1 - c0;
            lt.sign = 1.0;
            terms.push_back(lt);
          }
          tgs.push_back(T);
          tl.push_back(terms);
        }
        std::vector<int> where = emit_lflush(tgs, tl, tol);
        for (size_t q = 0; q < comps.size(); ++q) {
          if (P.ltg[where[q]].ws != nullptr) throw DeviceError("internal: dense compression outside the fused kernel");
          comps[q].T.rank = P.ltg[where[q]].info + 1;
        }
      }
      if (!comps.empty()) {
        // rewrite those dense terms as low-rank terms on the compressed factors
        size_t q = 0;
        for (auto& kv : pending) {
          HMat* C = kv.first.first;
          const LeafDesc& d = C->L[kv.first.second];
          if (d.kind != K_LR) continue;
          for (auto& pt : kv.second) {
            if (!pt.t.dense) continue;
            const Comp& c = comps[q++];
            pt.t.dense = 0;
            pt.t.U = c.T.U;
            pt.t.ldu = c.T.m;
            pt.t.W = c.T.V;
            pt.t.ldw = c.T.n;
            pt.t.k = c.T.rank;
            pt.kcap = c.kc;
          }
        }
      }
    }
    // the dense products and their compressions (steps 2-3) use none of the
    // applies' data (step 1): they run on the side stream while the applies
    // run, i.e. [products, compressions] forked, then the applies, then join
    if (ph_apply != (size_t)-1 && ph_dprod == ph_apply + 1) {
      const int chain = (int)(P.ph.size() - ph_dprod);
      std::rotate(P.ph.begin() + ph_apply, P.ph.begin() + ph_apply + 1, P.ph.end());
      P.ph[ph_apply].side = chain;
      P.ph[ph_apply].par = 1;
    }
    // 4. dense targets: their flushes join the first fused rounded-addition
    //    launch of step 5 (disjoint leaves), else get a phase of their own
    Phase dph{PH_DFLUSH, (int)P.dflush.size(), 0, 0, 0, 0, 0, 0.0};
    {
      for (auto& kv : pending) {
        HMat* C = kv.first.first;
        const LeafDesc& d = C->L[kv.first.second];
        if (d.kind != K_DENSE) continue;
        DFlushItem it{d.A, d.m, d.m, d.n, (int)P.terms.size(), (int)kv.second.size(), 0};
        for (auto& pt : kv.second) P.terms.push_back(pt.t);
        P.dflush.push_back(it);
      }
      dph.n0 = (int)P.dflush.size() - dph.b0;
    }
    const size_t ph_lr0 = P.ph.size();
    bool has_fused = false;
    // 5. low-rank targets: rounded additions, terms split so that the
    //    concatenated width stays within KMAX
    {
      // whole-list fused targets first, in a launch of their own (it may
      // overlap the rounds of the other targets), then the rounds
      std::vector<std::vector<std::pair<LFlushTarget, std::vector<Term>>>> rounds(1);
      for (auto& kv : pending) {
        HMat* C = kv.first.first;
        int leaf = kv.first.second;
        const LeafDesc& d = C->L[leaf];
        if (d.kind != K_LR) continue;
        if (fused_target(d, kv.second)) {
          // one fused target with the whole term list (dense terms were
          // compressed to low-rank temporaries above)
          LFlushTarget T{};
          T.U = d.A;
          T.V = d.B;
          T.rank = C->rank + leaf;
          T.m = d.m;
          T.n = d.n;
          T.kcap = d.kcap;
          T.Kcap = fused_width(tol);
          std::vector<Term> tl;
          for (auto& pt : kv.second) tl.push_back(pt.t);
          rounds[0].push_back({T, tl});
          continue;
        }
        // with double-double parts the fast core takes 48 columns: terms
        // wider than 48 - kcap are split into column pieces that fit
        std::vector<PendingTerm> split;
        const std::vector<PendingTerm>* tl_src = &kv.second;
        if (radd_dd(tol) && d.kcap <= 32) {
          const int w = 48 - d.kcap;
          for (const PendingTerm& pt : kv.second) {
            if (pt.kcap <= w || pt.t.dense != 0 || pt.t.klim > 0) {
              split.push_back(pt);
              continue;
            }
            for (int c0 = 0; c0 < pt.kcap; c0 += w) {
              PendingTerm sp = pt;
              sp.t.U = pt.t.U + (size_t)pt.t.ldu * c0;
              sp.t.W = pt.t.W + (size_t)pt.t.ldw * c0;
              sp.t.kofs = c0;
              sp.t.klim = std::min(w, pt.kcap - c0);
              sp.kcap = sp.t.klim;
              split.push_back(sp);
            }
          }
          tl_src = &split;
        }
        const std::vector<PendingTerm>& tsrc = *tl_src;
        size_t q = 0, rd = 0;
        while (q < tsrc.size()) {
          LFlushTarget T{};
          T.U = d.A;
          T.V = d.B;
          T.rank = C->rank + leaf;
          T.m = d.m;
          T.n = d.n;
          T.kcap = d.kcap;
          int K = d.kcap;
          // concatenations of at most 48 columns use the faster core kernel
          // (without double-double parts it takes KMAX)
          const int lim = radd_dd(tol) ? 48 : KMAX;
          std::vector<Term> tl;
          while (q < tsrc.size() && (K + tsrc[q].kcap <= lim || tl.empty())) {
            K += tsrc[q].kcap;
            tl.push_back(tsrc[q].t);
            ++q;
          }
          if (K > KMAX) throw DeviceError("internal: term wider than a rounded addition");
          T.Kcap = K;
          if (rounds.size() <= rd + 1) rounds.resize(rd + 2);
          rounds[rd + 1].push_back({T, tl});
          ++rd;
        }
      }
      has_fused = !rounds[0].empty();
      for (auto& r : rounds) {
        if (r.empty()) continue;
        std::vector<LFlushTarget> tgs;
        std::vector<std::vector<Term>> tl;
        for (auto& e : r) {
          tgs.push_back(e.first);
          tl.push_back(e.second);
        }
        emit_lflush(tgs, tl, tol);
      }
    }
    if (dph.n0) {
      if (P.ph.size() > ph_lr0 && P.ph[ph_lr0].type == PH_RADD) {
        P.ph[ph_lr0].b1 = dph.b0;
        P.ph[ph_lr0].n1 = dph.n0;
      } else {
        P.ph.insert(P.ph.begin() + ph_lr0, dph);
      }
    }
    // the whole-list fused targets (the first phase of step 5 when there
    // are any) and the rounds of the other targets write different leaves:
    // the fused launch overlaps the rounds
    if (has_fused && P.ph.size() > ph_lr0 + 1) {
      P.ph[ph_lr0].side = 1;
      P.ph[ph_lr0].par = (int)(P.ph.size() - ph_lr0 - 1);
    }
    bjobs.clear();
    bjob_mat.clear();
    bdprod.clear();
    pending.clear();
    for (auto& k : pkeys) k.first->pend[k.second] = -1;
    pkeys.clear();
    pterms.clear();
    if (!keep_ws) ws.release(mk);
    in_batch = false;
    if (after_batch && !in_defer && !keep_ws) after_batch();
    return mk;
  }

  void release_kept(const WsStack::Mark& m) { ws.release(m); }
  void phase_marker(int type) {
    P.ph.push_back(Phase{type, 0, 0, 0, 0, 0, 0, 0.0});
    if (type == PH_DEFER_BEGIN) in_defer = true;
    if (type == PH_DEFER_END) in_defer = false;
  }

  // Copies of leaves (add_copies) between copy_begin() and copy_end() go to
  // one phase.
  int copy_begin() const { return (int)P.copies.size(); }
  void copy_end(int b0) {
    Phase ph{PH_COPY, b0, (int)P.copies.size() - b0, 0, 0, 0, 0, 0.0};
    if (ph.n0) P.ph.push_back(ph);
  }

  // Copies the leaves of `node` of src (null: zeros) into dst, scaled;
  // add_identity_diag adds I to dense diagonal leaves; skip_compress leaves
  // out low-rank destinations of dense sources; move clears the source.
  void add_copies(HMat* dst, HMat* src, int node, double scale, bool add_identity_diag, bool skip_compress,
                  bool move) {
    const Structure& S = *dst->S;
    const BNode& b = S.bn[node];
    for (int l = b.lbeg; l < b.lend; ++l) {
      const LeafDesc& d = dst->L[l];
      if (d.kind == K_ZERO) continue;
      if (skip_compress && src && d.kind == K_LR && src->L[l].kind == K_DENSE) continue;
      CopyItem c{};
      c.dense = d.kind == K_DENSE;
      c.m = d.m;
      c.n = d.n;
      c.kcap = d.kcap;
      c.dA = d.A;
      c.dB = d.B;
      c.drank = d.kind == K_LR ? dst->rank + l : nullptr;
      if (src) {
        const LeafDesc& e = src->L[l];
        c.A = e.A;
        c.B = e.B;
        c.rank = e.kind == K_LR ? src->rank + l : nullptr;
        c.expand = (d.kind == K_DENSE && e.kind == K_LR) ? 1 : 0;
        if (d.kind == K_LR && e.kind != K_LR) throw DeviceError("internal: dense to low-rank copy");
        if (move) {
          if (c.expand) throw DeviceError("internal: move with expansion");
          if (e.kind == K_DENSE) c.zA = e.A;
          if (e.kind == K_LR) c.zrank = src->rank + l;
        }
      }
      c.scale = scale;
      c.add_identity = (add_identity_diag && S.lf[l].r == S.lf[l].c) ? 1 : 0;
      P.copies.push_back(c);
    }
  }

};

// H-LU of a diagonal block with the H-inverses of both factors (App. B.3
// recursion; inverses by the 2x2 block formulas):
//   LU(A11);  U12 = L11^{-1} A12;  L21 = A21 U11^{-1};  LU(A22 - L21 U12);
//   (L^{-1})21 = -L22^{-1} L21 L11^{-1};  (U^{-1})12 = -U11^{-1} U12 U22^{-1}.
// T21 = L21 L11^{-1} and S12 = U11^{-1} U12 are formed together with the
// Schur update, so that each level takes three batches of products.
struct LuCtx {
  HMat *LU, *Li, *Ui, *TMP;
};
struct LuNode {
  const LuCtx* c;
  int node;
};

// A diagonal node that is one dense leaf, or 2 x 2 dense leaves of at most
// LUINV_N rows in all, is factored with its inverses by one fused kernel.
static bool luinv_item(const LuCtx& c, int node, LuInvItem* out) {
  const Structure& S = *c.LU->S;
  const HMat *LU = c.LU, *Li = c.Li, *Ui = c.Ui;
  const BNode& b = S.bn[node];
  if (S.cl[b.r].hi - S.cl[b.r].lo > LUINV_N) return false;
  LuInvItem it{};
  if (b.kind != K_H) {
    const int l = b.leaf;
    if (LU->L[l].kind != K_DENSE || Li->L[l].kind != K_DENSE || Ui->L[l].kind != K_DENSE) return false;
    it.A11 = LU->L[l].A;
    it.L11 = Li->L[l].A;
    it.U11 = Ui->L[l].A;
    it.m1 = LU->L[l].m;
    it.m2 = 0;
  } else {
    int lf[4];
    for (int q = 0; q < 4; ++q) {
      const BNode& ch = S.bn[b.child[q]];
      if (ch.kind == K_H || LU->L[ch.leaf].kind != K_DENSE) return false;
      lf[q] = ch.leaf;
    }
    // Li: 11, 21, 22 dense (12 structurally zero); Ui: 11, 12, 22 dense
    if (Li->L[lf[0]].kind != K_DENSE || Li->L[lf[2]].kind != K_DENSE || Li->L[lf[3]].kind != K_DENSE ||
        Ui->L[lf[0]].kind != K_DENSE || Ui->L[lf[1]].kind != K_DENSE || Ui->L[lf[3]].kind != K_DENSE)
      return false;
    it.A11 = LU->L[lf[0]].A;
    it.A12 = LU->L[lf[1]].A;
    it.A21 = LU->L[lf[2]].A;
    it.A22 = LU->L[lf[3]].A;
    it.L11 = Li->L[lf[0]].A;
    it.L21 = Li->L[lf[2]].A;
    it.L22 = Li->L[lf[3]].A;
    it.U11 = Ui->L[lf[0]].A;
    it.U12 = Ui->L[lf[1]].A;
    it.U22 = Ui->L[lf[3]].A;
    it.m1 = LU->L[lf[0]].m;
    it.m2 = LU->L[lf[3]].m;
  }
  if (out) *out = it;
  return true;
}

// levels of the recursion below a diagonal node (0: factored by one kernel)
static int lu_height(const LuCtx& c, int node) {
  const BNode& b = c.LU->S->bn[node];
  if (b.kind != K_H || luinv_item(c, node, nullptr)) return 0;
  return 1 + std::max(lu_height(c, b.child[0]), lu_height(c, b.child[3]));
}

// The recursion over several diagonal nodes at once (of one or of several
// problems), aligned from the bottom: the nodes of height H take the three
// batches of their level together, and nodes of smaller height wait inside
// the first sub-recursion until their own level comes.  With one node this
// is the plain recursion.
static void hluinv_joint(Builder& B, const std::vector<LuNode>& items, int H) {
  if (items.empty()) return;
  if (H == 0) {
    Phase pl{PH_LUINV, (int)B.P.luinv.size(), 0, 0, 0, 0, 0, 0.0};
    std::vector<GetrfItem> gi;
    for (const LuNode& it : items) {
      LuInvItem li;
      if (luinv_item(*it.c, it.node, &li)) {
        B.P.luinv.push_back(li);
        continue;
      }
      const BNode& b = it.c->LU->S->bn[it.node];
      const LeafDesc& d = it.c->LU->L[b.leaf];
      gi.push_back(GetrfItem{d.A, it.c->Li->L[b.leaf].A, it.c->Ui->L[b.leaf].A, d.m, 0});
    }
    pl.n0 = (int)B.P.luinv.size() - pl.b0;
    if (pl.n0) B.P.ph.push_back(pl);
    if (!gi.empty()) {
      B.P.ph.push_back(Phase{PH_GETRF, (int)B.P.getrf.size(), (int)gi.size(), 0, 0, 0, 0, 0.0});
      for (auto& g : gi) B.P.getrf.push_back(g);
    }
    return;
  }
  std::vector<LuNode> act, sub;
  for (const LuNode& it : items) (lu_height(*it.c, it.node) == H ? act : sub).push_back(it);
  for (const LuNode& a : act) sub.push_back({a.c, a.c->LU->S->bn[a.node].child[0]});
  hluinv_joint(B, sub, H - 1);
  // TMP blocks start (and are left by the move below) at zero
  B.begin();
  for (const LuNode& a : act) {
    const BNode& b = a.c->LU->S->bn[a.node];
    const int n11 = b.child[0], n12 = b.child[1], n21 = b.child[2];
    const LuCtx& c = *a.c;
    B.mma(c.TMP, n12, c.Li, n11, c.LU, n12, 1.0);   // U12 = L11^{-1} A12
    B.mma(c.TMP, n21, c.LU, n21, c.Ui, n11, 1.0);   // L21 = A21 U11^{-1}
  }
  B.end();
  const int cb = B.copy_begin();
  for (const LuNode& a : act) {
    const BNode& b = a.c->LU->S->bn[a.node];
    for (int q : {1, 2}) B.add_copies(a.c->LU, a.c->TMP, b.child[q], 1.0, false, false, /*move=*/true);
  }
  B.copy_end(cb);
  B.begin();
  for (const LuNode& a : act) {
    const BNode& b = a.c->LU->S->bn[a.node];
    const int n12 = b.child[1], n21 = b.child[2], n22 = b.child[3];
    const LuCtx& c = *a.c;
    B.mma(c.LU, n22, c.LU, n21, c.LU, n12, -1.0);   // A22 -= L21 U12
  }
  B.end();
  // T21 and S12 are needed only after the recursion on A22 and touch none of
  // its blocks (they read L21, U12 and the inverses of node 11, and write the
  // TMP blocks 21 and 12): they run on the deferred stream meanwhile, their
  // workspace kept until the join
  B.phase_marker(PH_DEFER_BEGIN);
  B.begin();
  for (const LuNode& a : act) {
    const BNode& b = a.c->LU->S->bn[a.node];
    const int n11 = b.child[0], n12 = b.child[1], n21 = b.child[2];
    const LuCtx& c = *a.c;
    B.mma(c.TMP, n21, c.LU, n21, c.Li, n11, 1.0);   // T21 = L21 L11^{-1}
    B.mma(c.TMP, n12, c.Ui, n11, c.LU, n12, 1.0);   // S12 = U11^{-1} U12
  }
  const WsStack::Mark kept = B.end(/*keep_ws=*/true);
  B.phase_marker(PH_DEFER_END);
  std::vector<LuNode> sub2;
  for (const LuNode& a : act) sub2.push_back({a.c, a.c->LU->S->bn[a.node].child[3]});
  hluinv_joint(B, sub2, H - 1);
  B.phase_marker(PH_DEFER_JOIN);
  B.begin();
  for (const LuNode& a : act) {
    const BNode& b = a.c->LU->S->bn[a.node];
    const int n12 = b.child[1], n21 = b.child[2], n22 = b.child[3];
    const LuCtx& c = *a.c;
    B.mma(c.Li, n21, c.Li, n22, c.TMP, n21, -1.0);  // (L^{-1})21 = -L22^{-1} T21
    B.mma(c.Ui, n12, c.TMP, n12, c.Ui, n22, -1.0);  // (U^{-1})12 = -S12 U22^{-1}
  }
  B.end();
  B.release_kept(kept);
}

// Per-step matrix-vector plan of one H-matrix: projection tiles, the
// per-leaf-cluster entry lists and (optionally) FP32 copies of the factors.
struct MvPlan {
  DevBuf dtiles, dents, drows, dpart, f32pool, bf16pool;
  MvDev dev{};
  int64_t matrix_bytes = 0;   // stored bytes read per product
  int64_t lr_bytes = 0, dense_bytes = 0;
  int64_t u_bytes = 0, v_bytes = 0;   // low-rank factors read by the gather / the projection
  int64_t lr_entries = 0, dense_entries = 0;
  int64_t nslots = 0;

  // lr_fmt: storage of the low-rank leaves (MV_FMT_F64, _F32 or _BF16),
  // except those with at most lr64_rows rows and columns, which stay FP64;
  // force_kb: the rank bucket (0: chosen from the ranks below); gather_waves:
  // wavefronts per gather workgroup (0: 8 single-problem, 4 batched)
  void create(const Structure& S, const HMat& M, const std::vector<int32_t>& rk, bool dense_f32, int lr_fmt,
              hipStream_t s, int force_kb = 0, int gather_waves = 0, int lr64_rows = 0) {
    const double* base = M.mem;
    const float* fbase = nullptr;
    const uint16_t* hbase = nullptr;
    if (dense_f32 || lr_fmt == MV_FMT_F32) {
      f32pool.alloc(std::max<size_t>(M.pool_doubles, 1) * sizeof(float));
      HL_CHECK(launch_convert_f32(base, f32pool.as<float>(), M.pool_doubles, s));
      fbase = f32pool.as<float>();
    }
    if (lr_fmt == MV_FMT_BF16) {
      bf16pool.alloc(std::max<size_t>(M.pool_doubles, 1) * sizeof(uint16_t));
      HL_CHECK(launch_convert_bf16(base, bf16pool.as<uint16_t>(), M.pool_doubles, s));
      hbase = bf16pool.as<uint16_t>();
    }
    auto fptr = [&](const double* p) -> const void* { return fbase + (p - base); };
    const size_t d_elt = dense_f32 ? sizeof(float) : sizeof(double);
    // format of a low-rank leaf, its element size and the address of a value
    auto leaf_fmt = [&](const LeafDesc& d) {
      return std::max(d.m, d.n) > lr64_rows ? lr_fmt : (int)MV_FMT_F64;
    };
    auto fmt_elt = [](int f) { return f == MV_FMT_F64 ? sizeof(double) : (f == MV_FMT_F32 ? sizeof(float) : 2); };
    auto lr_ptr = [&](int f, const double* p) -> const void* {
      if (f == MV_FMT_F32) return fptr(p);
      if (f == MV_FMT_BF16) return hbase + (p - base);
      return p;
    };
    // rank bucket kb: 8 when leaves of higher rank (split below into
    // kb-column chunks, each with its own tiles, partial slots and gather
    // entries) add at most 50 % more low-rank entries, else 16 when they add
    // at most 10 %, else 32.  A few ranks just above a bucket then cost an
    // extra narrow entry instead of moving every entry to the wider kernels.
    int kmax = 0;
    int64_t nlr = 0, extra8 = 0, extra16 = 0;
    for (size_t l = 0; l < S.lf.size(); ++l)
      if (M.L[l].kind == K_LR && rk[l] > 0) {
        kmax = std::max(kmax, rk[l]);
        ++nlr;
        extra8 += (rk[l] + 7) / 8 - 1;
        extra16 += (rk[l] + 15) / 16 - 1;
      }
    if (kmax > 32) throw std::runtime_error("internal: rank above 32 in a product plan");
    const int kb = force_kb ? force_kb : (2 * extra8 <= nlr ? 8 : (10 * extra16 <= nlr ? 16 : 32));
    // projection tiles: a leaf's V rows split into at most MV_PMAX tiles of
    // whole passes; partial slots of one leaf are consecutive
    std::vector<MvTile> tiles;
    std::vector<int32_t> slot0(S.lf.size(), 0), np(S.lf.size(), 0);
    for (size_t l = 0; l < S.lf.size(); ++l) {
      const LeafDesc& d = M.L[l];
      if (d.kind == K_DENSE) {
        dense_bytes += (int64_t)d.m * d.n * d_elt;
        dense_entries += (int64_t)d.m * d.n;
      }
      if (d.kind != K_LR || rk[l] == 0) continue;
      const int k = rk[l];
      const int fmt = leaf_fmt(d);
      const size_t lr_elt = fmt_elt(fmt);
      const int rpp = project_rows_per_pass(kb, fmt != MV_FMT_F64);
      lr_bytes += (int64_t)(d.m + d.n) * k * lr_elt;
      u_bytes += (int64_t)d.m * k * lr_elt;
      v_bytes += (int64_t)d.n * k * lr_elt;
      lr_entries += (int64_t)(d.m + d.n) * k;
      const int npass = (d.n + rpp - 1) / rpp;
      const int per = (npass + MV_PMAX - 1) / MV_PMAX;   // passes per tile
      const int P = (npass + per - 1) / per;
      slot0[l] = (int32_t)nslots;
      np[l] = P;
      // chunk ch (columns ch kb .. ch kb + kc - 1) owns slots slot0 + ch P ..
      const int nch = (k + kb - 1) / kb;
      for (int ch = 0; ch < nch; ++ch) {
        const int kc = std::min(kb, k - ch * kb);
        for (int t = 0; t < P; ++t) {
          const int r0 = t * per * rpp, r1 = std::min(d.n, r0 + per * rpp);
          // one tile per project_width(kb) columns
          const int tw = project_width(kb);
          for (int c0 = 0; c0 < kc; c0 += tw) {
            MvTile T{};
            T.n = r1 - r0;
            T.k = std::min(kc - c0, tw);
            T.ld = d.n;
            T.xoff = d.clo + r0;
            T.slot = (int32_t)(nslots + ch * P + t);
            T.f32 = fmt;
            T.col0 = c0;
            const double* p = d.B + r0 + (size_t)d.n * (ch * kb + c0);
            T.V = lr_ptr(fmt, p);
            tiles.push_back(T);
          }
        }
      }
      nslots += (int64_t)nch * P;
    }
    matrix_bytes = dense_bytes + lr_bytes;
    // longest tiles first
    std::stable_sort(tiles.begin(), tiles.end(), [](const MvTile& a, const MvTile& b) { return a.n > b.n; });
    std::vector<MvEntry> ents;
    std::vector<MvRow> rows;
    std::vector<std::pair<int64_t, MvEntry>> row;
    for (size_t q = 0; q < S.leafcl.size(); ++q) {
      const Cluster& c = S.cl[S.leafcl[q]];
      row.clear();
      for (int e = S.rowptr[q]; e < S.rowptr[q + 1]; ++e) {
        const int l = S.rowidx[e];
        const LeafDesc& d = M.L[l];
        if (d.kind == K_DENSE) {
          // pieces of MV_DCOLS columns: the wavefronts of the gather share
          // a dense leaf instead of one of them streaming all its columns
          for (int c0 = 0; c0 < d.n; c0 += MV_DCOLS) {
            MvEntry D{};
            D.kind = 0;
            D.n = std::min(MV_DCOLS, d.n - c0);
            D.xoff = d.clo + c0;
            D.ld = d.m;
            const double* p = d.A + (c.lo - d.rlo) + (size_t)d.m * c0;
            D.ptr = dense_f32 ? fptr(p) : (const void*)p;
            row.emplace_back((int64_t)D.n * d_elt, D);
          }
        } else if (d.kind == K_LR && rk[l] > 0) {
          // one entry per kb-column chunk of the factor
          const int fmt = leaf_fmt(d);
          for (int ch = 0; ch * kb < rk[l]; ++ch) {
            MvEntry L{};
            L.kind = fmt == MV_FMT_F64 ? 1 : (fmt == MV_FMT_F32 ? 2 : 3);
            L.n = np[l];
            L.k = std::min(kb, rk[l] - ch * kb);
            L.slot = slot0[l] + ch * np[l];
            L.ld = d.m;
            const double* p = d.A + (c.lo - d.rlo) + (size_t)d.m * ch * kb;
            L.ptr = lr_ptr(fmt, p);
            row.emplace_back((int64_t)L.k * (int64_t)fmt_elt(fmt), L);
          }
        }
      }
      // most bytes first: the wavefronts take entries round-robin
      std::stable_sort(row.begin(), row.end(),
                       [](const std::pair<int64_t, MvEntry>& a, const std::pair<int64_t, MvEntry>& b) {
                         return a.first > b.first;
                       });
      MvRow R{c.lo, c.hi, (int)ents.size(), 0};
      for (auto& pe : row) ents.push_back(pe.second);
      R.eend = (int)ents.size();
      rows.push_back(R);
    }
    upload(dtiles, tiles, s);
    upload(dents, ents, s);
    upload(drows, rows, s);
    dpart.alloc(std::max<int64_t>(nslots, 1) * kb * sizeof(double));
    dev = MvDev{dtiles.as<MvTile>(), dents.as<MvEntry>(), drows.as<MvRow>(), dpart.as<double>(),
                (int)tiles.size(), (int)rows.size(), kb, dense_f32 ? 1 : 0,
                gather_waves ? gather_waves : 8, gather_waves ? gather_waves : 4};
  }
  void run(const double* x, const MvEpi& e, hipStream_t s) const { HL_CHECK(mv_launch(dev, x, e, s)); }
};

// Bytes MvPlan::create allocates for a matrix of layout M with every
// low-rank leaf at rank kcap (the most it can hold), maximised over the
// rank buckets the plan may choose: an upper bound of the actual plan.
static size_t mvplan_bytes_bound(const Structure& S, const HMat& M, int lr_fmt) {
  const bool f32 = lr_fmt != MV_FMT_F64;   // narrow storage: the passes of a projection tile
  auto round8 = [](size_t b) { return std::max<size_t>(b, 8); };
  size_t best = 0;
  for (int kb : {8, 16, 32}) {
    int64_t ntiles = 0, nents = 0, nslots = 0;
    std::vector<int32_t> np(S.lf.size(), 0);
    for (size_t l = 0; l < S.lf.size(); ++l) {
      const LeafDesc& d = M.L[l];
      if (d.kind != K_LR || d.kcap == 0) continue;
      const int k = d.kcap;
      const int rpp = project_rows_per_pass(kb, f32);
      const int npass = (d.n + rpp - 1) / rpp;
      const int per = (npass + MV_PMAX - 1) / MV_PMAX;
      const int P = (npass + per - 1) / per;
      np[l] = P;
      const int nch = (k + kb - 1) / kb;
      const int tw = project_width(kb);
      for (int ch = 0; ch < nch; ++ch) {
        const int kc = std::min(kb, k - ch * kb);
        ntiles += (int64_t)P * ((kc + tw - 1) / tw);
      }
      nslots += (int64_t)nch * P;
    }
    for (size_t q = 0; q < S.leafcl.size(); ++q)
      for (int e = S.rowptr[q]; e < S.rowptr[q + 1]; ++e) {
        const LeafDesc& d = M.L[S.rowidx[e]];
        if (d.kind == K_DENSE) nents += (d.n + MV_DCOLS - 1) / MV_DCOLS;
        else if (d.kind == K_LR && d.kcap > 0) nents += (d.kcap + kb - 1) / kb;
      }
    size_t b = round8(ntiles * sizeof(MvTile)) + round8(nents * sizeof(MvEntry)) +
               round8(S.leafcl.size() * sizeof(MvRow)) + (size_t)std::max<int64_t>(nslots, 1) * kb * sizeof(double);
    best = std::max(best, b);
  }
  // the FP32 copy (dense leaves of the mixed paths, low-rank leaves in FP32)
  // and the BF16 copy of the pool
  if (f32) best += std::max<size_t>(M.pool_doubles, 1) * sizeof(float);
  if (lr_fmt == MV_FMT_BF16) best += std::max<size_t>(M.pool_doubles, 1) * sizeof(uint16_t);
  return best;
}

// Resident bytes of an operator (G with its structure lists, product plan
// and work vectors) and of one factor (the inverse factors, their product
// plans with FP32 copies on the mixed path, the G plan and work vectors):
// the allocations of assemble_ops and factor_group, with every low-rank
// block at its rank capacity.
static int prec_lr_fmt(int prec) {
  return prec == HLEVY_PREC_FP64 ? MV_FMT_F64 : (prec == HLEVY_PREC_MIXED ? MV_FMT_F32 : MV_FMT_BF16);
}

static size_t footprint_bytes(const Structure& S, int kcap, int prec) {
  auto round8 = [](size_t b) { return std::max<size_t>(b, 8); };
  const size_t P = S.leafcl.size(), nl = S.lf.size(), N = S.N;
  auto hmat = [&](const HMat& t) {
    return round8(t.pool_doubles * sizeof(double)) + round8(nl * sizeof(LeafDesc)) + round8(nl * sizeof(int32_t));
  };
  size_t b = 0;
  // structure lists, point maps, constants, overflow counter
  b += 2 * round8((P + 1) * 4) + round8(S.rowidx.size() * 4) + round8(S.colidx.size() * 4) + 2 * round8(P * 4) +
       2 * round8(N * 4) + 64 * 64 * sizeof(double) + 7 * sizeof(double) + 8;
  if (!S.var_s.empty())   // variable order: values, kernel constants, quadrature constants, row map
    b += 2 * round8(S.var_s.size() * 8) + round8(S.var_s.size() * 5 * 8) + round8(N * 4);
  HMat g;
  g.layout(S, kcap, FULL, false);
  b += hmat(g) + 2 * N * sizeof(double) + mvplan_bytes_bound(S, g, MV_FMT_F64);
  // the factor
  HMat li, ui;
  li.layout(S, kcap, LOWER, false);
  ui.layout(S, kcap, UPPER, false);
  b += hmat(li) + hmat(ui) + 7 * N * sizeof(double);
  b += mvplan_bytes_bound(S, g, MV_FMT_F64) + mvplan_bytes_bound(S, li, prec_lr_fmt(prec)) +
       mvplan_bytes_bound(S, ui, prec_lr_fmt(prec));
  return b;
}

// Products with one matrix kind (G, L^{-1} or U^{-1}) of every problem of a
// batch: problems grouped by rank bucket, dense precision and member bound
// (1, 2 or the most a launch takes), one projection and one gather launch
// per group.  Tiles and leaf clusters of the problems are interleaved, so
// each launch's work is spread over the whole chip.
struct MvBatch {
  struct Group {
    int kb, f32, rmax, gwb, w0, nw, r0, nr;
  };
  std::vector<Group> groups;
  DevBuf dw, dr;
  void create(const std::vector<const MvPlan*>& plans, const std::vector<int>& nrs, hipStream_t s) {
    std::map<std::tuple<int, int, int, int>, std::vector<int>> by;
    for (size_t i = 0; i < plans.size(); ++i) {
      const int kb = plans[i]->dev.kb;
      const int rb = nrs[i] <= 1 ? 1 : (nrs[i] <= 2 ? 2 : mv_batch_rmax(kb));
      if (nrs[i] > rb) throw DeviceError("internal: too many members in a batched problem");
      by[{kb, plans[i]->dev.dense_f32, rb, plans[i]->dev.gwb}].push_back((int)i);
    }
    std::vector<MvRef> w, r;
    for (auto& kv : by) {
      Group g{std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
              (int)w.size(), 0, (int)r.size(), 0};
      int tmax = 0, rmax = 0;
      for (int i : kv.second) {
        tmax = std::max(tmax, plans[i]->dev.ntiles);
        rmax = std::max(rmax, plans[i]->dev.nrows);
      }
      for (int t = 0; t < tmax; ++t)
        for (int i : kv.second)
          if (t < plans[i]->dev.ntiles) w.push_back(MvRef{i, 0, plans[i]->dev.tiles + t});
      for (int q = 0; q < rmax; ++q)
        for (int i : kv.second)
          if (q < plans[i]->dev.nrows) r.push_back(MvRef{i, 0, plans[i]->dev.rows + q});
      g.nw = (int)w.size() - g.w0;
      g.nr = (int)r.size() - g.r0;
      groups.push_back(g);
    }
    upload(dw, w, s);
    upload(dr, r, s);
  }
  void run(const MvInst* inst, int step, hipStream_t s) const {
    for (const Group& g : groups)
      HL_CHECK(mv_batch_launch(inst, dw.as<MvRef>() + g.w0, g.nw, dr.as<MvRef>() + g.r0, g.nr, g.kb, g.f32 != 0,
                               g.rmax, g.gwb, step, s));
  }
};

static MvEpi epi_plain(double* y) {
  MvEpi e{};
  e.kind = MV_EPI_PLAIN;
  e.y = y;
  return e;
}

static std::vector<int32_t> read_ranks(const HMat& M, hipStream_t s) {
  std::vector<int32_t> rk(M.L.size());
  if (!rk.empty())
    HL_CHECK(hipMemcpyAsync(rk.data(), M.rank, rk.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  HL_CHECK(hipStreamSynchronize(s));
  return rk;
}

}  // namespace hl

using namespace hl;

// Scratch of hlevy_solve_noalloc: the four work vectors, the two check slots
// and the check partial sums of one single-column solve.  Each device holds
// its own copy until the process ends.  Host code never uses the array's
// name as an address: the device address is taken with hipGetSymbolAddress,
// once per device (assembly is the set-up call), and kept here.
static constexpr size_t kScratchDoubles = 4 * (size_t)HLEVY_NOALLOC_MAX_N + 2 + 2 * 256;
static __device__ __align__(256) double scratch[kScratchDoubles];
static std::mutex g_scratch_mu;
static std::map<int, double*> g_scratch_ptr;   // device ordinal -> address of `scratch` there

// Device address of `scratch` on the current device (resolved on the first
// call per device).
static double* scratch_ptr() {
  int dev = 0;
  HL_CHECK(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* p = nullptr;
  HL_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw DeviceError("hipGetSymbolAddress returned no address for the scratch array");
  g_scratch_ptr.emplace(dev, static_cast<double*>(p));
  return static_cast<double*>(p);
}

struct hlevy_op {
  size_t bytes = 0;    // resident device bytes (declared first: freed last)
  AllocCtx actx{};     // the caller's allocator and this handle's byte counter
  hlevy_problem prob{};
  hlevy_hparams hp{};
  Structure S;
  ProblemDev pd{};
  DevStructure ds;
  HMat G;
  DevBuf cst, ovf;
  DevBuf var_s, var_C, var_cst, var_row;   // variable-order kernel (ProblemDev)
  DevBuf xbuf, ybuf;   // cluster-order work vectors for hlevy_matvec
  MvPlan mv;           // FP64 product with G
};

struct hlevy_fac {
  size_t bytes = 0;    // resident device bytes (declared first: freed last)
  AllocCtx actx{};     // the operator's allocator and this handle's byte counter
  const hlevy_op* op = nullptr;
  double dt = 0, lu_tol = 0;
  int prec = 0;
  HMat LU, Li, Ui;
  DevBuf w_u, w_y, w_b, w_z, w_r, w_d, w_g;
  MvPlan mvG, mvLi, mvUi;
  int32_t rank_overflows = 0;
};

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

template <class F>
static hlevy_status guarded(F&& f) {
  try {
    return f();
  } catch (const DeviceError& e) {
    return fail(HLEVY_ERR_DEVICE, e.msg);
  } catch (const OomError& e) {
    return fail(HLEVY_ERR_OOM, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(HLEVY_ERR_OOM, "host allocation failed");
  } catch (...) {
    return fail(HLEVY_ERR_DEVICE, "unexpected exception");
  }
}

static double frac_constant(int d, double s) {
  return std::pow(4.0, s) * std::tgamma(d / 2.0 + s) / (std::pow(M_PI, d / 2.0) * std::fabs(std::tgamma(-s)));
}

// Device slots of the residual checks of a call: (||r||^2, ||b||^2) per
// check, plus the partial sums of the norm kernels (reused in stream order).
struct CheckBuf {
  DevBuf slots, partial;
  int cap = 0;
  void reserve(int count, int N) {
    cap = std::max(count, 1);
    slots.alloc((size_t)2 * cap * sizeof(double));
    partial.alloc((size_t)2 * check_blocks(N) * sizeof(double));
  }
  double* slot(int i) const { return slots.as<double>() + 2 * (size_t)i; }
  // waits for the stream
  std::vector<double> read(int count, hipStream_t s) const {
    std::vector<double> v((size_t)2 * count);
    if (count > 0)
      HL_CHECK(hipMemcpyAsync(v.data(), slots.p, v.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HL_CHECK(hipStreamSynchronize(s));
    return v;
  }
};
static double rel_residual(double r2, double b2) {
  if (b2 > 0.0) return std::sqrt(r2 / b2);
  return r2 > 0.0 ? INFINITY : 0.0;
}

// One problem advanced by step_states: its factor, its vectors (cluster
// order: u^n, the iterate w, two temporaries), optionally its own
// projection partial buffers for G, L^{-1}, U^{-1} (null: the plans' own;
// problems that share a factor in one batch need buffers of their own) and
// its number of steps (negative: all steps of the call).
// check: the state's last step measures the relative residual of its
// final iterate (one more product with G) into *rel (host).
struct StepState {
  hlevy_fac* f;
  double *uc, *w, *z, *r;
  double *partG, *partL, *partU;
  int64_t steps = -1;
  bool check = false;
  double* rel = nullptr;
};

// Unforced Crank-Nicolson steps of every state (hlevy_step's recursion:
// M w = 2 u^n, u^{n+1} = w - u^n, `sweeps` refinement sweeps), each product
// one batched launch pair over all states.  States of one factor that have
// partial buffers of their own are taken as members of one batched problem
// (up to the launch's member bound, longest remaining first), so that their
// products read the factor once.  The last step of a checking state runs
// after the loop, with every checking state together: its last sweep
// updates w (the same arithmetic as the fused update of u^{n+1}), the
// residual of w is measured, then u^{n+1} = w - u^n.  Synchronises `s`
// before return (the tables are freed here).
static void step_states(const std::vector<StepState>& st, int64_t nsteps, int sweeps, hipStream_t s) {
  if (st.empty() || nsteps == 0) return;
  if (nsteps > INT32_MAX) throw DeviceError("internal: too many steps in one batched call");
  auto steps_of = [&](const StepState& x) {
    return (int32_t)(x.steps < 0 ? nsteps : std::min<int64_t>(x.steps, nsteps));
  };
  // problems: lists of member states
  std::vector<std::vector<int>> probs;
  {
    std::map<hlevy_fac*, std::vector<int>> byfac;
    std::vector<hlevy_fac*> order;
    for (size_t i = 0; i < st.size(); ++i) {
      const StepState& x = st[i];
      if (!x.partG || !x.partL || !x.partU) {
        probs.push_back({(int)i});   // uses the plans' own partial buffers: alone
        continue;
      }
      if (!byfac.count(x.f)) order.push_back(x.f);
      byfac[x.f].push_back((int)i);
    }
    for (hlevy_fac* f : order) {
      std::vector<int>& v = byfac[f];
      std::stable_sort(v.begin(), v.end(), [&](int a, int b) { return steps_of(st[a]) > steps_of(st[b]); });
      const int rm = std::min({mv_batch_rmax(f->mvG.dev.kb), mv_batch_rmax(f->mvLi.dev.kb),
                               mv_batch_rmax(f->mvUi.dev.kb), MV_RMAX});
      for (size_t q = 0; q < v.size(); q += rm)
        probs.emplace_back(v.begin() + q, v.begin() + std::min(v.size(), q + rm));
    }
  }
  std::vector<const MvPlan*> pg, pl, pu;
  std::vector<int> nrs;
  for (auto& pr : probs) {
    hlevy_fac* f = st[pr[0]].f;
    pg.push_back(&f->mvG);
    pl.push_back(&f->mvLi);
    pu.push_back(&f->mvUi);
    nrs.push_back((int)pr.size());
  }
  MvBatch bG, bL, bU;
  bG.create(pg, nrs, s);
  bL.create(pl, nrs, s);
  bU.create(pu, nrs, s);
  enum { T_AXPY, T_SUB, T_W, T_RES, T_LI, T_ADD, T_NEXT, T_COUNT };
  // tab: the loop (a checking state's last step left out); fin: the last
  // step of the checking states (the others sit out)
  std::vector<std::vector<MvInst>> tab(T_COUNT), fin(T_COUNT);
  bool any_check = false;
  for (const StepState& x : st) any_check = any_check || (x.check && steps_of(x) > 0);
  for (auto& pr : probs) {
    hlevy_fac* f = st[pr[0]].f;
    std::vector<MvInst> t(T_COUNT);
    for (int k = 0; k < T_COUNT; ++k) {
      t[k] = MvInst{};
      t[k].nr = (int32_t)pr.size();
      t[k].dev = (k == T_RES) ? f->mvG.dev : ((k == T_AXPY || k == T_LI) ? f->mvLi.dev : f->mvUi.dev);
    }
    for (size_t m = 0; m < pr.size(); ++m) {
      const StepState& x = st[pr[m]];
      double* pG = x.partG ? x.partG : f->mvG.dev.part;
      double* pL = x.partL ? x.partL : f->mvLi.dev.part;
      double* pU = x.partU ? x.partU : f->mvUi.dev.part;
      for (int k = 0; k < T_COUNT; ++k) {
        t[k].steps[m] = steps_of(x) - (x.check && steps_of(x) > 0 ? 1 : 0);
        t[k].part[m] = (k == T_RES) ? pG : ((k == T_AXPY || k == T_LI) ? pL : pU);
        t[k].epi[m] = MvEpi{};
      }
      // z = 2 L^{-1} u^n
      t[T_AXPY].x[m] = x.uc;
      t[T_AXPY].epi[m].kind = MV_EPI_AXPY;
      t[T_AXPY].epi[m].hdt = 2.0;
      t[T_AXPY].epi[m].y = x.z;
      // u^{n+1} = U^{-1} z - u^n
      t[T_SUB].x[m] = x.z;
      t[T_SUB].epi[m].kind = MV_EPI_SUB;
      t[T_SUB].epi[m].u = x.uc;
      t[T_SUB].epi[m].y = x.uc;
      // w = U^{-1} z
      t[T_W].x[m] = x.z;
      t[T_W].epi[m] = epi_plain(x.w);
      // r = 2 u^n - (w - dt/2 G w)
      t[T_RES].x[m] = x.w;
      t[T_RES].epi[m].kind = MV_EPI_CNRES;
      t[T_RES].epi[m].hdt = 0.5 * f->dt;
      t[T_RES].epi[m].u = x.uc;
      t[T_RES].epi[m].b = x.w;
      t[T_RES].epi[m].y = x.r;
      // z = L^{-1} r
      t[T_LI].x[m] = x.r;
      t[T_LI].epi[m] = epi_plain(x.z);
      // w += U^{-1} z
      t[T_ADD].x[m] = x.z;
      t[T_ADD].epi[m].kind = MV_EPI_ADD;
      t[T_ADD].epi[m].u = x.w;
      t[T_ADD].epi[m].y = x.w;
      // u^{n+1} = w + U^{-1} z - u^n
      t[T_NEXT].x[m] = x.z;
      t[T_NEXT].epi[m].kind = MV_EPI_NEXT;
      t[T_NEXT].epi[m].b = x.w;
      t[T_NEXT].epi[m].u = x.uc;
      t[T_NEXT].epi[m].y = x.uc;
    }
    for (int k = 0; k < T_COUNT; ++k) {
      tab[k].push_back(t[k]);
      for (size_t m = 0; m < pr.size(); ++m) {
        const StepState& x = st[pr[m]];
        t[k].steps[m] = (x.check && steps_of(x) > 0) ? 1 : 0;
      }
      fin[k].push_back(t[k]);
    }
  }
  std::vector<DevBuf> dtab(T_COUNT), dfin(T_COUNT);
  for (int k = 0; k < T_COUNT; ++k) upload(dtab[k], tab[k], s);
  if (any_check)
    for (int k = 0; k < T_COUNT; ++k) upload(dfin[k], fin[k], s);
  auto T = [&](int k) { return dtab[k].as<MvInst>(); };
  auto F = [&](int k) { return dfin[k].as<MvInst>(); };
  for (int64_t n = 0; n < nsteps; ++n) {
    const int k = (int)n;
    bL.run(T(T_AXPY), k, s);
    if (sweeps == 0) {
      bU.run(T(T_SUB), k, s);
      continue;
    }
    bU.run(T(T_W), k, s);
    for (int it = 0; it < sweeps; ++it) {
      bG.run(T(T_RES), k, s);
      bL.run(T(T_LI), k, s);
      bU.run(T(it + 1 < sweeps ? T_ADD : T_NEXT), k, s);
    }
  }
  if (any_check) {
    // the checking states' last step: w by `sweeps` updates, the residual
    // of w, its norms, then u^{n+1} = w - u^n
    bL.run(F(T_AXPY), 0, s);
    bU.run(F(T_W), 0, s);
    for (int it = 0; it < sweeps; ++it) {
      bG.run(F(T_RES), 0, s);
      bL.run(F(T_LI), 0, s);
      bU.run(F(T_ADD), 0, s);
    }
    bG.run(F(T_RES), 0, s);
    std::vector<int> chk;
    int nmax = 1;
    for (size_t i = 0; i < st.size(); ++i)
      if (st[i].check && steps_of(st[i]) > 0) {
        chk.push_back((int)i);
        nmax = std::max(nmax, st[i].f->op->S.N);
      }
    CheckBuf cb;
    cb.reserve((int)chk.size(), nmax);
    for (size_t q = 0; q < chk.size(); ++q) {
      const StepState& x = st[chk[q]];
      const int N = x.f->op->S.N;
      HL_CHECK(launch_check_norms(x.r, x.uc, 2.0, nullptr, 0.0, N, cb.partial.as<double>(), cb.slot((int)q), s));
      HL_CHECK(launch_wsub(x.uc, x.w, N, s));
    }
    const std::vector<double> v = cb.read((int)chk.size(), s);
    for (size_t q = 0; q < chk.size(); ++q)
      if (st[chk[q]].rel) *st[chk[q]].rel = rel_residual(v[2 * q], v[2 * q + 1]);
  }
  // the tables and maps are freed on return: wait for the device first
  HL_CHECK(hipStreamSynchronize(s));
}

// Factorisation memory (bytes) of one problem while it is being factored:
// the LU workspace, the workspace inverse factors and the temporary (leaf-
// level blocks dense), the final inverse factors and, roughly, the product
// workspace of the recursion.
static constexpr size_t kDefaultFactorWorkspace = (size_t)48 << 30;

static size_t factor_footprint(const hlevy_op& op) {
  const int kc = op.hp.max_rank;
  HMat t;
  size_t d = 0;
  d += 2 * t.layout(op.S, kc, FULL, true);
  d += t.layout(op.S, kc, LOWER, true) + t.layout(op.S, kc, UPPER, true);
  d += t.layout(op.S, kc, LOWER, false) + t.layout(op.S, kc, UPPER, false);
  return d * sizeof(double) + (d * sizeof(double)) / 2;
}

// H-LU with inverse factors of every problem of `fs` in one plan: the
// recursion runs jointly over the problems (hluinv_joint), so each batch of
// products, copies and rounded additions is one launch for all of them.
// Problems share the zero-pivot flag and the rank-overflow counter of the
// group.
static hlevy_status factor_group(std::vector<hlevy_fac*>& fs, Arena& arena, WsStack& ws, hipStream_t s) {
  const double lu_tol = fs[0]->lu_tol;
  const int prec = fs[0]->prec;
  struct Work {
    HMat Li, Ui, TMP;
    LuCtx ctx;
  };
  std::vector<std::unique_ptr<Work>> wk;
  DevBuf zpb, ovfb;
  zpb.alloc(sizeof(int32_t));
  ovfb.alloc(sizeof(int32_t));
  HL_CHECK(hipMemsetAsync(zpb.p, 0, sizeof(int32_t), s));
  HL_CHECK(hipMemsetAsync(ovfb.p, 0, sizeof(int32_t), s));
  const double ta = now_s();
  {
    size_t need = 0;
    for (hlevy_fac* f : fs) {
      HMat t;
      const size_t nl = f->op->S.lf.size();
      const int kc = f->op->hp.max_rank;
      // LU and TMP full, L^{-1} lower, U^{-1} upper: the two triangles can
      // differ when the rank cap subdivided a block but not its transpose
      need += 2 * HMat::arena_bytes(t.layout(f->op->S, kc, FULL, true), nl);
      need += HMat::arena_bytes(t.layout(f->op->S, kc, LOWER, true), nl);
      need += HMat::arena_bytes(t.layout(f->op->S, kc, UPPER, true), nl);
    }
    arena.reserve(need);
  }
  const WsStack::Mark ws0 = ws.mark();
  for (hlevy_fac* f : fs) {
    const Structure& S = f->op->S;
    const int kc = f->op->hp.max_rank;
    const bool dmax = true;   // leaf-level admissible blocks dense while factoring
    auto w = std::make_unique<Work>();
    // workspaces in the arena (LU too: the per-step path needs only G and
    // the inverse factors)
    f->LU.create_in(arena, S, kc, FULL, s, dmax);
    w->Li.create_in(arena, S, kc, LOWER, s, dmax);
    w->Ui.create_in(arena, S, kc, UPPER, s, dmax);
    w->TMP.create_in(arena, S, kc, FULL, s, dmax);
    {
      AllocScope own(&f->actx);
      f->Li.create(S, kc, LOWER, s);
      f->Ui.create(S, kc, UPPER, s);
    }
    w->ctx = LuCtx{&f->LU, &w->Li, &w->Ui, &w->TMP};
    wk.push_back(std::move(w));
  }
  HL_CHECK(hipStreamSynchronize(s));
  const double t0 = now_s();
  double tpost = 0.0;
  {
    Plan P;
    Builder B(P, ws, fs[0]->op->ds.ident.as<double>(), ovfb.as<int32_t>(), lu_tol);
    for (hlevy_fac* f : fs) B.add_problem(f->op->S, f->op->ds);
    int cb = B.copy_begin();
    for (hlevy_fac* f : fs)   // M = I - dt/2 G
      B.add_copies(&f->LU, const_cast<HMat*>(&f->op->G), 0, -0.5 * f->dt, true, false, false);
    B.copy_end(cb);
    cb = B.copy_begin();
    for (auto& w : wk)
      for (HMat* z : {&w->Li, &w->Ui, &w->TMP}) B.add_copies(z, nullptr, 0, 0.0, false, false, false);
    B.copy_end(cb);
    std::vector<LuNode> roots;
    int H = 0;
    for (auto& w : wk) {
      roots.push_back({&w->ctx, 0});
      H = std::max(H, lu_height(w->ctx, 0));
    }
    // The plan goes to the device in segments at batch boundaries while the
    // rest is being built, so the device starts after the first segment's
    // planning instead of the whole plan's.  Segments run in order on the
    // same streams as one plan would (the deferred stream's join and the
    // workspace reuse keep their order); each stays alive until the end.
    std::vector<std::unique_ptr<Plan>> segs;
    size_t next_flush = 64;
    auto launch_segment = [&]() {
      ForkJoin& fj = fork_join();
      P.upload_all(fj.upload);
      HL_CHECK(hipEventRecord(fj.uploaded, fj.upload));
      HL_CHECK(hipStreamWaitEvent(s, fj.uploaded, 0));
      P.run(zpb.as<int32_t>(), s);
    };
    B.after_batch = [&]() {
      if (P.ph.size() < next_flush) return;
      launch_segment();
      segs.push_back(std::make_unique<Plan>());
      P.swap_contents(*segs.back());
      next_flush = 1536;
    };
    hluinv_joint(B, roots, H);
    B.after_batch = nullptr;
    // inverse factors in the operator's block format: dense leaf-level
    // blocks of the workspace are truncated back to low rank
    cb = B.copy_begin();
    for (size_t q = 0; q < fs.size(); ++q)
      for (int side = 0; side < 2; ++side)
        B.add_copies(side == 0 ? &fs[q]->Li : &fs[q]->Ui, side == 0 ? &wk[q]->Li : &wk[q]->Ui, 0, 1.0, false,
                     /*skip_compress=*/true, false);
    B.copy_end(cb);
    // one target per block with its dense content as 32-column terms (the
    // targets start at rank 0; without double-double parts a 64-column
    // block is one concatenation, with them the fused kernel takes the
    // pieces in two)
    std::vector<LFlushTarget> tgs;
    std::vector<std::vector<Term>> tl;
    for (size_t q = 0; q < fs.size(); ++q)
      for (int side = 0; side < 2; ++side) {
        const HMat& src = side == 0 ? wk[q]->Li : wk[q]->Ui;
        HMat& dst = side == 0 ? fs[q]->Li : fs[q]->Ui;
        for (size_t l = 0; l < dst.L.size(); ++l) {
          const LeafDesc& d = dst.L[l];
          if (!(d.kind == K_LR && src.L[l].kind == K_DENSE)) continue;
          LFlushTarget T{};
          T.U = d.A;
          T.V = d.B;
          T.rank = dst.rank + l;
          T.m = d.m;
          T.n = d.n;
          T.kcap = d.kcap;
          T.Kcap = fused_width(lu_tol);
          T.borth = 1;
          std::vector<Term> terms;
          const int w = d.kcap <= 16 ? 32 : 16;   // kcap + w <= 48
          if (d.kcap > 32) throw DeviceError("internal: rank capacity above 32");
          for (int c0 = 0; c0 < d.n; c0 += w) {
            const int c1 = std::min(d.n, c0 + w);
            Term tm{};
            tm.dense = 0;
            tm.ro = 0;
            tm.mr = d.m;
            tm.co = c0;
            tm.nc = c1 - c0;
            tm.U = src.L[l].A + (size_t)d.m * c0;
            tm.ldu = d.m;
            tm.W = B.ident;
            tm.ldw = 64;
            tm.kfix = c1 - c0;
            tm.sign = 1.0;
            terms.push_back(tm);
          }
          tgs.push_back(T);
          tl.push_back(terms);
        }
      }
    B.emit_lflush(tgs, tl, lu_tol);
    const double t1 = now_s();
    const double t2 = t1;
    launch_segment();
    const double t3 = now_s();
    HL_CHECK(hipStreamSynchronize(s));
    const double t4 = now_s();
    if (verbose())
      std::fprintf(stderr, "[hlevy] factor %zu problem(s): alloc %.3fs plan+early segments %.3fs (%zu segments "
                   "before the last: its %zu phases, %zu lr targets, ws peak %.1f MB) upload %.3fs enqueue %.3fs "
                   "device-tail %.3fs\n", fs.size(), t0 - ta, t1 - t0, segs.size(), P.ph.size(), P.ltg.size(),
                   ws.peak / 1048576.0, t2 - t1, t3 - t2, t4 - t3);
    tpost = now_s();
  }
  int32_t zp = 0, ovf = 0;
  HL_CHECK(hipMemcpy(&zp, zpb.p, sizeof(int32_t), hipMemcpyDeviceToHost));
  HL_CHECK(hipMemcpy(&ovf, ovfb.p, sizeof(int32_t), hipMemcpyDeviceToHost));
  if (zp) return fail(HLEVY_ERR_ZERO_PIVOT, "zero pivot in a diagonal leaf of the H-LU");
  // A rounded addition truncated at the rank capacity leaves the factors
  // less accurate than lu_tol says.  Such overflows are reported
  // (hlevy_fac_info, stats) and the refinement's residual checks guard the
  // solutions; operators assembled with strict_rank_cap refuse FP64 factors
  // that overflow (the direct solver must then meet lu_tol).
  bool strict = false;
  for (hlevy_fac* f : fs) strict = strict || f->op->hp.strict_rank_cap;
  if (ovf > 0 && prec == HLEVY_PREC_FP64 && strict)
    return fail(HLEVY_ERR_RANK_CAP, std::to_string(ovf) + " rounded additions of the FP64 H-LU needed more than "
                                        "the rank capacity (raise max_rank or lu_tol, or factor in mixed precision)");
  const bool mixed = prec != HLEVY_PREC_FP64;
  const int lr_fmt = prec_lr_fmt(prec);
  for (hlevy_fac* f : fs) {
    f->rank_overflows = ovf;
    const Structure& S = f->op->S;
    const size_t Nb = (size_t)S.N * sizeof(double);
    AllocScope own(&f->actx);
    for (DevBuf* b : {&f->w_u, &f->w_y, &f->w_b, &f->w_z, &f->w_r, &f->w_d, &f->w_g}) b->alloc(Nb);
    // residual operator in FP64 on both paths: with the far field in FP32
    // the operator applied to smooth states is off by ~1e-7 relative (the
    // far-field sums are large and cancel against the near field), which
    // adds up to ~1e-8..1e-7 over 1000 steps; preconditioner (inverse
    // factors): FP32 on the mixed paths, with BF16 low-rank leaves on the
    // BF16 one
    const hlevy_hparams& hp = f->op->hp;
    f->mvG.create(S, f->op->G, read_ranks(f->op->G, s), false, MV_FMT_F64, s, hp.rank_bucket, hp.gather_waves);
    f->mvLi.create(S, f->Li, read_ranks(f->Li, s), mixed, lr_fmt, s, hp.rank_bucket, hp.gather_waves);
    f->mvUi.create(S, f->Ui, read_ranks(f->Ui, s), mixed, lr_fmt, s, hp.rank_bucket, hp.gather_waves);
    // the LU's storage is the arena's, reused by the next group
    f->LU.L.clear();
    f->LU.mem = nullptr;
    f->LU.ldev = nullptr;
    f->LU.rank = nullptr;
  }
  ws.release(ws0);
  HL_CHECK(hipStreamSynchronize(s));
  if (verbose())
    std::fprintf(stderr, "[hlevy] factor %zu problem(s): workspace free + product plans %.3fs\n", fs.size(),
                 now_s() - tpost);
  return HLEVY_OK;
}

extern "C" {

int32_t hlevy_abi_version(void) { return HLEVY_ABI_VERSION; }

const char* hlevy_last_error(void) { return g_last_error.c_str(); }

hlevy_status hlevy_plan_info(const hlevy_problem* prob, const hlevy_hparams* hp, hlevy_plan_info_t* out) {
  if (!prob || !hp || !out) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  try {
    Structure S;
    std::string e = build_structure(*prob, *hp, S);
    if (!e.empty()) return fail(HLEVY_ERR_INVALID_ARG, e);
    out->N = S.N;
    out->depth = S.depth;
    out->n_clusters = (int32_t)S.cl.size();
    out->n_dense = S.n_dense;
    out->n_lowrank = S.n_lr;
    int mx = 0, mn = 1 << 30;
    for (int c : S.leafcl) {
      mx = std::max(mx, S.cl[c].hi - S.cl[c].lo);
      mn = std::min(mn, S.cl[c].hi - S.cl[c].lo);
    }
    out->max_leaf_points = mx;
    out->min_leaf_points = mn;
    out->dense_entries = S.dense_entries;
    return HLEVY_OK;
  } catch (const std::bad_alloc&) {
    return fail(HLEVY_ERR_OOM, "host allocation failed");
  }
}

}  // extern "C"

using SplitSet = std::set<std::pair<int32_t, int32_t>>;

// Assembly of `count` problems (hlevy_assemble_batched).  splits[i]: the
// admissible blocks of problem i not stored low rank.  After the truncation
// the per-block overflow counts come back; a problem with blocks whose
// compression needed more than the rank capacity is assembled again with
// those blocks subdivided (dense at the leaf level), until none overflows.
static hlevy_status assemble_ops(const hlevy_problem* probs, const hlevy_hparams* hps, const SplitSet* splits,
                                 int32_t count, const hlevy_allocator* al, hipStream_t s,
                                 std::vector<std::unique_ptr<hlevy_op>>& ops) {
  ops.clear();
  ops.resize(count);
  // 1. trees on the host; constants, near field and ACA of every problem
  //    enqueued back to back
  struct Aca {
    std::vector<int32_t> lr_ids;
    std::vector<int64_t> uo, vo;
    DevBuf buf, rank, dids, lids, duo, dvo, blkovf;
  };
  std::vector<std::unique_ptr<Aca>> aca(count);
  const int kaca = KMAX;
  for (int32_t i = 0; i < count; ++i) {
    const hlevy_problem* prob = probs + i;
    const hlevy_hparams* hp = hps + i;
    auto op = std::make_unique<hlevy_op>();
    if (al) op->actx.al = *al;
    op->actx.count = &op->bytes;
    std::string e = build_structure(*prob, *hp, op->S, splits ? &splits[i] : nullptr);
    if (!e.empty()) return fail(HLEVY_ERR_INVALID_ARG, e);
    const Structure& S = op->S;
    op->prob = *prob;
    op->prob.mask = nullptr;      // the caller's arrays: the structure keeps what it needs
    op->prob.s_field = nullptr;
    op->hp = *hp;
    ProblemDev& pd = op->pd;
    pd.dim = prob->dim;
    pd.n = prob->n;
    pd.N = S.N;
    pd.h = S.h;
    pd.a = prob->a;
    pd.b0 = prob->b[0];
    pd.b1 = prob->dim == 2 ? prob->b[1] : 0.0;
    pd.c = prob->c;
    pd.s = prob->s;
    pd.lam = prob->lambda;
    pd.kernel = prob->kernel;
    pd.eps2 = prob->eps2;
    pd.lam_neg = prob->lambda_neg;
    pd.C = prob->C > 0.0 ? prob->C : (prob->kernel == HLEVY_KERNEL_GAUSSIAN ? 1.0 : frac_constant(prob->dim, prob->s));
    pd.r0 = prob->r0;
    {
      AllocScope own(&op->actx);
      op->ds.create(S, s);
      op->cst.alloc(7 * sizeof(double));   // S0, S2, C2, T, S1 (+ S2, C2 of the second axis, 2D asymmetric)
      op->ovf.alloc(sizeof(int32_t));
      op->G.create(S, hp->max_rank, FULL, s);
    }
    HL_CHECK(hipMemsetAsync(op->ovf.p, 0, sizeof(int32_t), s));
    if (prob->kernel == HLEVY_KERNEL_VARIABLE_ORDER) {
      // constants of every distinct jump index; hlevy_op_constants reports
      // those of the first point (natural order)
      std::vector<double> vC(S.var_s.size());
      for (size_t q = 0; q < vC.size(); ++q) vC[q] = prob->C > 0.0 ? prob->C : frac_constant(prob->dim, S.var_s[q]);
      {
        AllocScope own(&op->actx);
        upload(op->var_s, S.var_s, s);
        upload(op->var_C, vC, s);
        upload(op->var_row, S.var_row, s);
        op->var_cst.alloc(5 * sizeof(double) * S.var_s.size());
      }
      pd.var_s = op->var_s.as<double>();
      pd.var_C = op->var_C.as<double>();
      pd.var_row = op->var_row.as<int32_t>();
      pd.var_cst = op->var_cst.as<double>();
      pd.nvar = (int32_t)S.var_s.size();
      HL_CHECK(launch_constants_var(pd, op->var_cst.as<double>(), s));
      int first = 0;
      for (int k = 0; k < S.N; ++k)
        if (S.perm[k] == 0) first = S.var_row[k];
      HL_CHECK(hipMemcpyAsync(op->cst.p, op->var_cst.as<double>() + 5 * (size_t)first, 5 * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    } else {
      HL_CHECK(launch_constants(pd, op->cst.as<double>(), s));
    }
    // dense near field
    auto A = std::make_unique<Aca>();
    std::vector<int32_t> dense_ids;
    for (size_t l = 0; l < S.lf.size(); ++l) (S.lf[l].kind == K_DENSE ? dense_ids : A->lr_ids).push_back((int)l);
    upload(A->dids, dense_ids, s);
    upload(A->lids, A->lr_ids, s);
    HL_CHECK(launch_fill_dense(pd, op->cst.as<double>(), op->ds.lat.as<int32_t>(), op->G.dev(),
                               A->dids.as<int32_t>(), (int)dense_ids.size(), s));
    if (hp->taylor_rank > 0) {
      // the fixed-rank Taylor factors of the Gaussian kernel (Sec. 3.3) go
      // straight into G: no ACA, no truncation.  Every low-rank leaf holds
      // taylor_rank columns (the structure keeps thinner blocks dense).
      for (int l : A->lr_ids)
        if (op->G.L[l].kcap < hp->taylor_rank) throw DeviceError("internal: a Taylor block above its rank capacity");
      HL_CHECK(launch_taylor(pd, op->ds.lat.as<int32_t>(), op->G.dev(), A->lids.as<int32_t>(),
                             (int)A->lr_ids.size(), op->G.rank, hp->taylor_rank, s));
      A->lr_ids.clear();
    }
    // far field: ACA into scratch (truncated into G below)
    int64_t tot = 0;
    for (int l : A->lr_ids) {
      A->uo.push_back(tot);
      tot += (int64_t)S.lf[l].m * kaca;
      A->vo.push_back(tot);
      tot += (int64_t)S.lf[l].n * kaca;
    }
    A->buf.alloc(std::max<int64_t>(tot, 1) * sizeof(double));
    upload(A->duo, A->uo, s);
    upload(A->dvo, A->vo, s);
    A->rank.alloc(std::max<size_t>(A->lr_ids.size(), 1) * sizeof(int32_t));
    // per-block overflow counts of the truncation
    A->blkovf.alloc(std::max<size_t>(A->lr_ids.size(), 1) * sizeof(int32_t));
    HL_CHECK(hipMemsetAsync(A->blkovf.p, 0, std::max<size_t>(A->lr_ids.size(), 1) * sizeof(int32_t), s));
    HL_CHECK(launch_aca(pd, op->ds.lat.as<int32_t>(), op->G.dev(), A->lids.as<int32_t>(), (int)A->lr_ids.size(),
                        A->buf.as<double>(), A->buf.as<double>(), A->duo.as<int64_t>(), A->dvo.as<int64_t>(),
                        A->rank.as<int32_t>(), kaca, 0.1 * hp->aca_tol, s));
    aca[i] = std::move(A);
    ops[i] = std::move(op);
  }
  // 2. truncation of every ACA block to its tolerance: one plan for all
  //    problems (problems of equal tolerance share launches).  The ACA
  //    ranks come back first (one synchronisation): with double-double
  //    parts the fast cores take 48 columns, so an ACA term of rank k is
  //    split into ceil(k / (48 - kcap)) column pieces, piece p of every
  //    block applied in round p.
  std::vector<std::vector<int32_t>> aca_rank(count);
  for (int32_t i = 0; i < count; ++i) {
    aca_rank[i].resize(aca[i]->lr_ids.size());
    if (!aca_rank[i].empty())
      HL_CHECK(hipMemcpyAsync(aca_rank[i].data(), aca[i]->rank.as<int32_t>(), aca_rank[i].size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost, s));
  }
  HL_CHECK(hipStreamSynchronize(s));
  {
    std::map<double, std::vector<int32_t>> by_tol;
    for (int32_t i = 0; i < count; ++i) by_tol[ops[i]->hp.aca_tol].push_back(i);
    Plan P;
    WsStack ws;
    Builder B(P, ws, ops[0]->ds.ident.as<double>(), ops[0]->ovf.as<int32_t>(), hps[0].aca_tol);
    for (auto& kv : by_tol) {
      const bool split = radd_dd(kv.first);
      std::vector<std::vector<LFlushTarget>> tgs(1);
      std::vector<std::vector<std::vector<Term>>> tl(1);
      std::vector<std::vector<int32_t*>> ovf(1);
      for (int32_t i : kv.second) {
        hlevy_op* op = ops[i].get();
        const Aca& A = *aca[i];
        for (size_t q = 0; q < A.lr_ids.size(); ++q) {
          const LeafDesc& d = op->G.L[A.lr_ids[q]];
          const int w = split ? std::min(kaca, 48 - d.kcap) : kaca;
          if (w <= 0) throw DeviceError("internal: rank capacity above 47 with double-double parts");
          const int kr = aca_rank[i][q];
          if (kr < 0 || kr > kaca) throw DeviceError("internal: ACA rank out of range");
          // at least one piece: a block of rank 0 is still truncated (to rank 0)
          const int kend = split ? std::max(kr, 1) : kaca;
          for (int c0 = 0, piece = 0; c0 < kend; c0 += w, ++piece) {
            LFlushTarget T{};
            T.U = d.A;
            T.V = d.B;
            T.rank = op->G.rank + A.lr_ids[q];
            T.m = d.m;
            T.n = d.n;
            T.kcap = d.kcap;
            const int kl = std::min(w, kend - c0);
            T.Kcap = split ? d.kcap + kl : kaca;
            Term t{};
            t.dense = 0;
            t.ro = 0;
            t.mr = d.m;
            t.co = 0;
            t.nc = d.n;
            t.U = A.buf.as<double>() + A.uo[q] + (size_t)d.m * c0;
            t.ldu = d.m;
            t.W = A.buf.as<double>() + A.vo[q] + (size_t)d.n * c0;
            t.ldw = d.n;
            t.k = A.rank.as<int32_t>() + q;
            t.sign = 1.0;
            if (split) {
              t.kofs = c0;
              t.klim = kl;
            }
            if ((int)tgs.size() <= piece) {
              tgs.resize(piece + 1);
              tl.resize(piece + 1);
              ovf.resize(piece + 1);
            }
            tgs[piece].push_back(T);
            tl[piece].push_back({t});
            ovf[piece].push_back(A.blkovf.as<int32_t>() + q);
          }
        }
      }
      for (size_t piece = 0; piece < tgs.size(); ++piece) {
        // each target counts its overflows in its block's own counter
        std::vector<int> where = B.emit_lflush(tgs[piece], tl[piece], kv.first);
        for (size_t q = 0; q < where.size(); ++q) P.ltg[where[q]].overflow = ovf[piece][q];
      }
    }
    P.upload_all(s);
    P.run(nullptr, s);
    HL_CHECK(hipStreamSynchronize(s));
  }
  // 3. blocks over the rank capacity: their problems are assembled again
  //    with those blocks subdivided
  std::vector<int32_t> redo;
  std::vector<SplitSet> redo_split;
  for (int32_t i = 0; i < count; ++i) {
    const Aca& A = *aca[i];
    std::vector<int32_t> bo(A.lr_ids.size(), 0);
    if (!bo.empty())
      HL_CHECK(hipMemcpy(bo.data(), A.blkovf.p, bo.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    SplitSet sp = ops[i]->S.split;
    bool more = false;
    for (size_t q = 0; q < bo.size(); ++q)
      if (bo[q] > 0) {
        const LeafInfo& li = ops[i]->S.lf[A.lr_ids[q]];
        more = sp.insert({li.r, li.c}).second || more;
      }
    if (more) {
      redo.push_back(i);
      redo_split.push_back(std::move(sp));
    }
  }
  if (!redo.empty()) {
    std::vector<hlevy_problem> rp;
    std::vector<hlevy_hparams> rh;
    for (int32_t i : redo) {
      rp.push_back(probs[i]);
      rh.push_back(hps[i]);
    }
    std::vector<std::unique_ptr<hlevy_op>> again;
    hlevy_status st = assemble_ops(rp.data(), rh.data(), redo_split.data(), (int32_t)redo.size(), al, s, again);
    if (st != HLEVY_OK) return st;
    for (size_t q = 0; q < redo.size(); ++q) {
      ops[redo[q]] = std::move(again[q]);
      aca[redo[q]].reset();
    }
  }
  // 4. ranks back in one round, then the per-step product plans
  std::vector<std::vector<int32_t>> rk(count);
  for (int32_t i = 0; i < count; ++i) {
    if (!aca[i]) continue;   // assembled again above
    rk[i].resize(ops[i]->G.L.size());
    if (!rk[i].empty())
      HL_CHECK(hipMemcpyAsync(rk[i].data(), ops[i]->G.rank, rk[i].size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                              s));
  }
  HL_CHECK(hipStreamSynchronize(s));
  for (int32_t i = 0; i < count; ++i) {
    if (!aca[i]) continue;
    hlevy_op* op = ops[i].get();
    AllocScope own(&op->actx);
    op->xbuf.alloc((size_t)op->S.N * sizeof(double));
    op->ybuf.alloc((size_t)op->S.N * sizeof(double));
    op->mv.create(op->S, op->G, rk[i], false, MV_FMT_F64, s, op->hp.rank_bucket, op->hp.gather_waves);
  }
  aca.clear();
  HL_CHECK(hipStreamSynchronize(s));
  return HLEVY_OK;
}

extern "C" {

hlevy_status hlevy_assemble(const hlevy_problem* prob, const hlevy_hparams* hp, const hlevy_allocator* al,
                            void* stream, hlevy_op** out) {
  if (!prob || !hp || !out) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  return hlevy_assemble_batched(prob, hp, 1, al, stream, out);
}

hlevy_status hlevy_assemble_batched(const hlevy_problem* probs, const hlevy_hparams* hps, int32_t count,
                                    const hlevy_allocator* al, void* stream, hlevy_op** out) {
  if (!probs || !hps || !out) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  if (count < 1) return fail(HLEVY_ERR_INVALID_ARG, "count must be >= 1");
  if (al && (!al->alloc || !al->free)) return fail(HLEVY_ERR_INVALID_ARG, "allocator needs alloc and free");
  for (int32_t i = 0; i < count; ++i) out[i] = nullptr;
  std::vector<std::unique_ptr<hlevy_op>> ops;
  hlevy_status st = guarded([&]() -> hlevy_status {
    hipStream_t s = as_stream(stream);
    HL_CHECK(init_kernel_attributes());
    (void)scratch_ptr();   // set-up of hlevy_solve_noalloc on this device
    // transient buffers of the call go through the caller's allocator too
    AllocCtx call{};
    if (al) call.al = *al;
    AllocScope sc(&call);
    return assemble_ops(probs, hps, nullptr, count, al, s, ops);
  });
  if (st != HLEVY_OK) return st;
  for (int32_t i = 0; i < count; ++i) out[i] = ops[i].release();
  return HLEVY_OK;
}

hlevy_status hlevy_footprint(const hlevy_problem* prob, const hlevy_hparams* hp, int32_t prec, size_t* bytes_out) {
  if (!prob || !hp || !bytes_out) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  if (prec != HLEVY_PREC_FP64 && prec != HLEVY_PREC_MIXED && prec != HLEVY_PREC_MIXED_BF16)
    return fail(HLEVY_ERR_INVALID_ARG, "bad precision");
  try {
    Structure S;
    std::string e = build_structure(*prob, *hp, S);
    if (!e.empty()) return fail(HLEVY_ERR_INVALID_ARG, e);
    *bytes_out = footprint_bytes(S, hp->max_rank, prec);
    return HLEVY_OK;
  } catch (const std::bad_alloc&) {
    return fail(HLEVY_ERR_OOM, "host allocation failed");
  }
}

hlevy_status hlevy_fac_info(const hlevy_fac* f, hlevy_fac_info_t* out, void* stream) {
  if (!f || !out) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  return guarded([&]() -> hlevy_status {
    std::memset(out, 0, sizeof(*out));
    out->device_bytes = f->bytes;
    out->rank_overflows = f->rank_overflows;
    int mx = 0;
    for (const HMat* M : {&f->Li, &f->Ui}) {
      std::vector<int32_t> rk(M->L.size());
      if (!rk.empty())
        HL_CHECK(hipMemcpyAsync(rk.data(), M->rank, rk.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                                as_stream(stream)));
      HL_CHECK(hipStreamSynchronize(as_stream(stream)));
      for (size_t l = 0; l < rk.size(); ++l)
        if (M->L[l].kind == K_LR) mx = std::max(mx, rk[l]);
    }
    out->max_rank = mx;
    const MvPlan* pl[3] = {&f->mvG, &f->mvLi, &f->mvUi};
    for (int w = 0; w < 3; ++w) out->product_bytes[w] = (double)pl[w]->matrix_bytes;
    out->lu_tol = f->lu_tol;
    out->dt = f->dt;
    out->prec = f->prec;
    return HLEVY_OK;
  });
}

hlevy_status hlevy_op_constants(const hlevy_op* op, double out[5], void* stream) {
  if (!op || !out) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  return guarded([&]() -> hlevy_status {
    HL_CHECK(hipMemcpyAsync(out, op->cst.p, 5 * sizeof(double), hipMemcpyDeviceToHost, as_stream(stream)));
    HL_CHECK(hipStreamSynchronize(as_stream(stream)));
    return HLEVY_OK;
  });
}

hlevy_status hlevy_exterior_forcing(const hlevy_op* op, const double* u_ext, double* g, void* stream) {
  if (!op || !u_ext || !g) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  if (op->prob.kernel == HLEVY_KERNEL_VARIABLE_ORDER)
    return fail(HLEVY_ERR_INVALID_ARG, "the exterior forcing takes a constant jump index");
  if (op->prob.kernel == HLEVY_KERNEL_GAUSSIAN)
    return fail(HLEVY_ERR_INVALID_ARG, "the exterior forcing follows the window scheme (tempered kernels)");
  if (op->S.N != (op->prob.dim == 1 ? op->prob.n : op->prob.n * op->prob.n))
    return fail(HLEVY_ERR_INVALID_ARG, "the exterior forcing needs the whole box (no mask)");
  const int n = op->prob.n;
  const size_t next = op->prob.dim == 1 ? 2 * (size_t)(n + 1) : (size_t)(3 * n + 2) * (3 * n + 2);
  const size_t N = op->S.N;
  if (g < u_ext + next && u_ext < g + N) return fail(HLEVY_ERR_INVALID_ARG, "u_ext and g must not overlap");
  return guarded([&]() -> hlevy_status {
    hipStream_t s = as_stream(stream);
    DevBuf tab;
    if (op->prob.dim == 1) {
      tab.alloc((2 * (size_t)(n + 1) + 1) * sizeof(double));
      HL_CHECK(launch_exterior(op->pd, op->cst.as<double>(), u_ext, tab.as<double>(), g, s));
    } else {
      tab.alloc((size_t)(2 * n + 3) * (2 * n + 3) * sizeof(double));
      HL_CHECK(launch_exterior2(op->pd, op->cst.as<double>(), u_ext, 3 * n + 2, n + 1, tab.as<double>(), g, s));
    }
    HL_CHECK(hipStreamSynchronize(s));
    return HLEVY_OK;
  });
}

hlevy_status hlevy_exterior_forcing_far(const hlevy_op* op, const double* u_ext, int32_t next, double tail_left,
                                        double tail_right, double* g, void* stream) {
  if (!op || !u_ext || !g) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  if (op->prob.kernel == HLEVY_KERNEL_VARIABLE_ORDER)
    return fail(HLEVY_ERR_INVALID_ARG, "the exterior forcing takes a constant jump index");
  if (op->prob.kernel == HLEVY_KERNEL_GAUSSIAN)
    return fail(HLEVY_ERR_INVALID_ARG, "the exterior forcing follows the window scheme (tempered kernels)");
  const int n = op->prob.n, dim = op->prob.dim;
  if (op->S.N != (dim == 1 ? n : n * n))
    return fail(HLEVY_ERR_INVALID_ARG, "the exterior forcing needs the whole box (no mask)");
  const int nmax = dim == 1 ? (1 << 26) : (1 << 13);
  if (next < n + 1 || next > nmax)
    return fail(HLEVY_ERR_INVALID_ARG, dim == 1 ? "next must lie in [n + 1, 2^26]" : "next must lie in [n + 1, 2^13]");
  if (!std::isfinite(tail_left) || !std::isfinite(tail_right)) return fail(HLEVY_ERR_INVALID_ARG, "non-finite tail");
  const size_t next_vals = dim == 1 ? 2 * (size_t)next : (size_t)(n + 2 * next) * (n + 2 * next);
  const size_t N = op->S.N;
  if (g < u_ext + next_vals && u_ext < g + N) return fail(HLEVY_ERR_INVALID_ARG, "u_ext and g must not overlap");
  return guarded([&]() -> hlevy_status {
    hipStream_t s = as_stream(stream);
    DevBuf tab, far;
    if (dim == 1) {
      // the window part from the n + 1 values of each side nearest the box
      // (contiguous in u_ext), then the far field added row by row
      tab.alloc((2 * (size_t)(n + 1) + 1) * sizeof(double));
      HL_CHECK(launch_exterior(op->pd, op->cst.as<double>(), u_ext + (next - (n + 1)), tab.as<double>(), g, s));
      far.alloc((2 * (size_t)(next - n) + 2) * sizeof(double));
      HL_CHECK(launch_far_field(op->pd, u_ext, next, tail_left, tail_right, far.as<double>(), g, s));
    } else {
      tab.alloc((size_t)(2 * n + 3) * (2 * n + 3) * sizeof(double));
      HL_CHECK(launch_exterior2(op->pd, op->cst.as<double>(), u_ext, n + 2 * next, next, tab.as<double>(), g, s));
      far.alloc(((size_t)(2 * next + 1) * (2 * next + 1) + 2) * sizeof(double));
      HL_CHECK(launch_far_field2(op->pd, u_ext, next, tail_left, tail_right, far.as<double>(), g, s));
    }
    HL_CHECK(hipStreamSynchronize(s));
    return HLEVY_OK;
  });
}

hlevy_status hlevy_op_info(const hlevy_op* op, hlevy_op_info_t* out, void* stream) {
  if (!op || !out) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  return guarded([&]() -> hlevy_status {
    std::vector<int32_t> rk(op->S.lf.size());
    int32_t ov = 0;
    HL_CHECK(hipMemcpyAsync(rk.data(), op->G.rank, rk.size() * sizeof(int32_t), hipMemcpyDeviceToHost,
                            as_stream(stream)));
    HL_CHECK(hipMemcpyAsync(&ov, op->ovf.p, sizeof(int32_t), hipMemcpyDeviceToHost, as_stream(stream)));
    HL_CHECK(hipStreamSynchronize(as_stream(stream)));
    int64_t de = 0, le = 0;
    int mx = 0;
    double sum = 0;
    int cnt = 0;
    for (size_t l = 0; l < op->S.lf.size(); ++l) {
      const LeafInfo& li = op->S.lf[l];
      if (li.kind == K_DENSE) de += (int64_t)li.m * li.n;
      else {
        le += (int64_t)(li.m + li.n) * rk[l];
        mx = std::max(mx, rk[l]);
        sum += rk[l];
        ++cnt;
      }
    }
    out->dense_entries = de;
    out->lowrank_entries = le;
    out->max_rank = mx;
    out->mean_rank = cnt ? sum / cnt : 0.0;
    out->rank_overflows = ov;
    out->device_bytes = op->bytes;
    out->subdivided_blocks = (int32_t)op->S.split.size();
    return HLEVY_OK;
  });
}

hlevy_status hlevy_matvec(const hlevy_op* op, const double* x, double* y, void* stream) {
  if (!op || !x || !y) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  if (x == y) return fail(HLEVY_ERR_INVALID_ARG, "x and y must not alias");
  return guarded([&]() -> hlevy_status {
    hipStream_t s = as_stream(stream);
    const int N = op->S.N;
    const int32_t* perm = op->ds.perm.as<int32_t>();
    HL_CHECK(launch_perm_gather(op->xbuf.as<double>(), x, perm, N, s));
    op->mv.run(op->xbuf.as<double>(), epi_plain(op->ybuf.as<double>()), s);
    HL_CHECK(launch_perm_scatter(y, op->ybuf.as<double>(), perm, N, s));
    return HLEVY_OK;
  });
}

hlevy_status hlevy_op_densify(const hlevy_op* op, double* dense, void* stream) {
  if (!op || !dense) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  return guarded([&]() -> hlevy_status {
    HL_CHECK(launch_densify(op->G.dev(), op->G.rank, (int)op->S.lf.size(), op->ds.perm.as<int32_t>(), op->S.N,
                            dense, as_stream(stream)));
    return HLEVY_OK;
  });
}

hlevy_status hlevy_factor(const hlevy_op* op, double dt, int32_t prec, double lu_tol, void* stream,
                          hlevy_fac** out) {
  if (!op || !out) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  return hlevy_factor_batched(&op, &dt, 1, prec, lu_tol, 0, stream, out);
}

hlevy_status hlevy_factor_batched(const hlevy_op* const* ops, const double* dt, int32_t count, int32_t prec,
                                  double lu_tol, size_t workspace_bytes, void* stream, hlevy_fac** out) {
  if (!ops || !dt || !out) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  if (count < 1) return fail(HLEVY_ERR_INVALID_ARG, "count must be >= 1");
  for (int32_t i = 0; i < count; ++i) {
    out[i] = nullptr;
    if (!ops[i]) return fail(HLEVY_ERR_INVALID_ARG, "null operator");
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return fail(HLEVY_ERR_INVALID_ARG, "dt must be > 0");
  }
  if (!(lu_tol > 0.0 && lu_tol < 1.0)) return fail(HLEVY_ERR_INVALID_ARG, "lu_tol must be in (0, 1)");
  if (prec != HLEVY_PREC_FP64 && prec != HLEVY_PREC_MIXED && prec != HLEVY_PREC_MIXED_BF16)
    return fail(HLEVY_ERR_INVALID_ARG, "bad precision");
  const size_t budget = workspace_bytes ? workspace_bytes : kDefaultFactorWorkspace;
  std::vector<std::unique_ptr<hlevy_fac>> fs(count);
  hlevy_status st = guarded([&]() -> hlevy_status {
    hipStream_t s = as_stream(stream);
    // transient buffers of the call: the first operator's allocator
    AllocCtx call{ops[0]->actx.al, nullptr};
    AllocScope sc(&call);
    for (int32_t i = 0; i < count; ++i) {
      fs[i] = std::make_unique<hlevy_fac>();
      fs[i]->actx = AllocCtx{ops[i]->actx.al, &fs[i]->bytes};
      fs[i]->op = ops[i];
      fs[i]->dt = dt[i];
      fs[i]->prec = prec;
      fs[i]->lu_tol = lu_tol;
    }
    // groups of consecutive problems whose factorisation memory fits the
    // budget; the groups share one arena and one product workspace
    Arena arena;
    WsStack ws;
    int32_t i0 = 0;
    while (i0 < count) {
      int32_t i1 = i0;
      size_t used = 0;
      while (i1 < count) {
        const size_t b = factor_footprint(*ops[i1]);
        if (i1 > i0 && used + b > budget) break;
        used += b;
        ++i1;
      }
      std::vector<hlevy_fac*> grp;
      for (int32_t i = i0; i < i1; ++i) grp.push_back(fs[i].get());
      hlevy_status e = factor_group(grp, arena, ws, s);
      if (e != HLEVY_OK) return e;
      i0 = i1;
    }
    return HLEVY_OK;
  });
  if (st != HLEVY_OK) return st;
  for (int32_t i = 0; i < count; ++i) out[i] = fs[i].release();
  return HLEVY_OK;
}

// Refinement sweeps when the caller gives none.  FP64 factors take one
// sweep too: products with the explicit inverse factors lose accuracy like
// eps * cond(L) * cond(U), which grows like N^2 on diffusion-dominated
// operators (about 1e-6 relative residual at N = 65536); one sweep with the
// FP64 operator brings the residual back to about 1e-12.
static int default_sweeps(const hlevy_fac* f, const hlevy_refine* refine) {
  if (refine) return refine->sweeps;
  return f->prec == HLEVY_PREC_FP64 ? 1 : 2;
}

static const char* refine_error(const hlevy_refine* r) {
  if (!r) return nullptr;
  if (r->sweeps < 0 || r->sweeps > 64) return "sweeps in [0, 64]";
  if (r->max_sweeps < 0 || r->max_sweeps > 64) return "max_sweeps in [0, 64]";
  if (r->check_every < 0) return "check_every must be >= 0";
  if (std::isnan(r->tol) || std::isinf(r->tol)) return "tol must be finite";
  return nullptr;
}

struct CheckLog {
  hlevy_stats* st;
  void begin(const hlevy_fac* f) {
    if (!st) return;
    std::memset(st, 0, sizeof(*st));
    st->last_rel_residual = -1.0;
    st->max_rel_residual = -1.0;
    st->rank_overflows = f->rank_overflows;
  }
  void note(double rel, int sweeps) {
    if (!st) return;
    st->checks++;
    st->last_rel_residual = rel;
    if (!(st->max_rel_residual >= rel)) st->max_rel_residual = rel;
    st->max_sweeps_used = std::max(st->max_sweeps_used, sweeps);
  }
};

// One right-hand side of hlevy_solve.  b, x: the caller's vectors (natural
// order); work: 4 N doubles (b, x, z, r in cluster order); chk: 2 check slots
// followed by 2 * check_blocks(N) partial sums (used when checking).  The
// products are those of the one-column solve: x = U^{-1} L^{-1} b, `sweeps`
// sweeps x += U^{-1} L^{-1} (b - M x), then at a check further sweeps while
// the relative residual misses tol, up to maxsw.  x is written only when the
// column is accepted.  Synchronises `s` only when checking.
static hlevy_status solve_column(hlevy_fac* f, const double* b, double* x, double* work, double* chk, int sweeps,
                                 double tol, int maxsw, bool checking, CheckLog& log, hipStream_t s) {
  const int N = f->op->S.N;
  const int32_t* perm = f->op->ds.perm.as<int32_t>();
  const double hdt = 0.5 * f->dt;
  double *qb = work, *qx = work + N, *qz = work + 2 * (size_t)N, *qr = work + 3 * (size_t)N;
  HL_CHECK(launch_perm_gather(qb, b, perm, N, s));
  MvEpi res{};               // r = b - (x - dt/2 G x)
  res.kind = MV_EPI_RESID;
  res.hdt = hdt;
  res.u = qx;
  res.b = qb;
  res.y = qr;
  MvEpi add{};               // x += U^{-1} z
  add.kind = MV_EPI_ADD;
  add.u = qx;
  add.y = qx;
  f->mvLi.run(qb, epi_plain(qz), s);
  f->mvUi.run(qz, epi_plain(qx), s);
  for (int it = 0; it < sweeps; ++it) {
    f->mvG.run(qx, res, s);
    f->mvLi.run(qr, epi_plain(qz), s);
    f->mvUi.run(qz, add, s);
  }
  if (checking) {
    int used = sweeps;
    for (;;) {
      f->mvG.run(qx, res, s);
      HL_CHECK(launch_check_norms(qr, qb, 1.0, nullptr, 0.0, N, chk + 2, chk, s));
      double v[2];
      HL_CHECK(hipMemcpyAsync(v, chk, sizeof(v), hipMemcpyDeviceToHost, s));
      HL_CHECK(hipStreamSynchronize(s));
      const double rel = rel_residual(v[0], v[1]);
      const bool ok = !(tol > 0.0) || rel <= tol;
      if (ok || used >= maxsw) {
        log.note(rel, used);
        if (!ok)
          return fail(HLEVY_ERR_NOT_CONVERGED, "refinement reached a relative residual of " + std::to_string(rel) +
                                                   " after " + std::to_string(used) + " sweeps (tol " +
                                                   std::to_string(tol) + ")");
        break;
      }
      f->mvLi.run(qr, epi_plain(qz), s);
      f->mvUi.run(qz, add, s);
      ++used;
    }
  }
  HL_CHECK(launch_perm_scatter(x, qx, perm, N, s));
  return HLEVY_OK;
}

hlevy_status hlevy_solve(hlevy_fac* f, const double* b, double* x, int64_t nrhs, int64_t ld,
                         const hlevy_refine* refine, hlevy_stats* stats, void* stream) {
  if (!f || !b || !x) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  const int64_t N = f->op->S.N;
  if (nrhs < 1) return fail(HLEVY_ERR_INVALID_ARG, "nrhs must be >= 1");
  if (ld < N) return fail(HLEVY_ERR_INVALID_ARG, "ld must be >= N");
  {
    const double* bl = b;
    const double* bh = b + (size_t)(nrhs - 1) * ld + N;
    const double* xl = x;
    const double* xh = x + (size_t)(nrhs - 1) * ld + N;
    if (bl < xh && xl < bh) return fail(HLEVY_ERR_INVALID_ARG, "b and x must not overlap");
  }
  if (const char* e = refine_error(refine)) return fail(HLEVY_ERR_INVALID_ARG, e);
  const double t_start = now_s();
  CheckLog log{stats};
  log.begin(f);
  return guarded([&]() -> hlevy_status {
    hipStream_t s = as_stream(stream);
    const int32_t* perm = f->op->ds.perm.as<int32_t>();
    const int sweeps = default_sweeps(f, refine);
    const double tol = refine ? refine->tol : 0.0;
    const int maxsw = std::max(sweeps, refine ? refine->max_sweeps : 0);
    const bool checking = stats || tol > 0.0;
    const double hdt = 0.5 * f->dt;
    // right-hand sides in groups of rm members of one batched problem:
    // every product reads the factor once for the whole group
    const int rm = nrhs == 1 ? 1
                             : std::min({mv_batch_rmax(f->mvG.dev.kb), mv_batch_rmax(f->mvLi.dev.kb),
                                         mv_batch_rmax(f->mvUi.dev.kb), MV_RMAX});
    const int R = (int)std::min<int64_t>(rm, nrhs);
    if (R == 1) {
      // one column at a time: the work vectors and the check slots of the
      // single-column solve
      DevBuf work;
      work.alloc((4 * (size_t)N + 2 + 2 * (size_t)check_blocks((int)N)) * sizeof(double));
      for (int64_t c = 0; c < nrhs; ++c) {
        const hlevy_status st = solve_column(f, b + (size_t)c * ld, x + (size_t)c * ld, work.as<double>(),
                                             work.as<double>() + 4 * (size_t)N, sweeps, tol, maxsw, checking, log, s);
        if (st != HLEVY_OK) {
          if (stats) {
            stats->steps_done = c;
            stats->seconds = now_s() - t_start;
          }
          return st;
        }
      }
      // the work vectors are freed on return: wait for the device first
      HL_CHECK(hipStreamSynchronize(s));
      if (stats) {
        stats->steps_done = nrhs;
        stats->seconds = now_s() - t_start;
      }
      return HLEVY_OK;
    }
    // per member: b, x, z, r in cluster order, and partial buffers
    const size_t nG = (size_t)std::max<int64_t>(f->mvG.nslots, 1) * f->mvG.dev.kb;
    const size_t nL = (size_t)std::max<int64_t>(f->mvLi.nslots, 1) * f->mvLi.dev.kb;
    const size_t nU = (size_t)std::max<int64_t>(f->mvUi.nslots, 1) * f->mvUi.dev.kb;
    const size_t per = 4 * (size_t)N + (R > 1 ? nG + nL + nU : 0);
    DevBuf work;
    work.alloc(per * R * sizeof(double));
    CheckBuf cb;
    if (checking) cb.reserve(R, (int)N);
    struct Mem { double *b, *x, *z, *r, *pG, *pL, *pU; };
    std::vector<Mem> mem(R);
    for (int m = 0; m < R; ++m) {
      double* p = work.as<double>() + per * m;
      mem[m] = Mem{p, p + N, p + 2 * N, p + 3 * N, nullptr, nullptr, nullptr};
      if (R > 1) {
        mem[m].pG = p + 4 * N;
        mem[m].pL = mem[m].pG + nG;
        mem[m].pU = mem[m].pL + nL;
      }
    }
    // the batched tables of a group (R > 1)
    enum { S_L0, S_U0, S_RES, S_L1, S_ADD, S_COUNT };
    MvBatch bG, bL, bU;
    if (R > 1) {
      bG.create({&f->mvG}, {R}, s);
      bL.create({&f->mvLi}, {R}, s);
      bU.create({&f->mvUi}, {R}, s);
    }
    std::vector<DevBuf> dtab(S_COUNT);
    int64_t written = 0;
    for (int64_t c0 = 0; c0 < nrhs; c0 += R) {
      const int nr = (int)std::min<int64_t>(R, nrhs - c0);
      for (int m = 0; m < nr; ++m)
        HL_CHECK(launch_perm_gather(mem[m].b, b + (size_t)(c0 + m) * ld, perm, (int)N, s));
      std::function<void(int)> run;   // runs product kind k for the group
      {
        std::vector<MvInst> t(S_COUNT);
        for (int k = 0; k < S_COUNT; ++k) {
          t[k] = MvInst{};
          t[k].nr = nr;
          t[k].dev = k == S_RES ? f->mvG.dev : ((k == S_L0 || k == S_L1) ? f->mvLi.dev : f->mvUi.dev);
          for (int m = 0; m < nr; ++m) {
            const Mem& q = mem[m];
            t[k].steps[m] = 1;
            t[k].part[m] = k == S_RES ? q.pG : ((k == S_L0 || k == S_L1) ? q.pL : q.pU);
            MvEpi e{};
            switch (k) {
              case S_L0: t[k].x[m] = q.b; e = epi_plain(q.z); break;
              case S_U0: t[k].x[m] = q.z; e = epi_plain(q.x); break;
              case S_RES:
                t[k].x[m] = q.x;
                e.kind = MV_EPI_RESID;
                e.hdt = hdt;
                e.u = q.x;
                e.b = q.b;
                e.y = q.r;
                break;
              case S_L1: t[k].x[m] = q.r; e = epi_plain(q.z); break;
              case S_ADD:
                t[k].x[m] = q.z;
                e.kind = MV_EPI_ADD;
                e.u = q.x;
                e.y = q.x;
                break;
            }
            t[k].epi[m] = e;
          }
        }
        for (int k = 0; k < S_COUNT; ++k) upload(dtab[k], std::vector<MvInst>{t[k]}, s);
        run = [&](int k) {
          const MvBatch& B = k == S_RES ? bG : ((k == S_L0 || k == S_L1) ? bL : bU);
          B.run(dtab[k].as<MvInst>(), 0, s);
        };
      }
      run(S_L0);
      run(S_U0);
      for (int it = 0; it < sweeps; ++it) {
        run(S_RES);
        run(S_L1);
        run(S_ADD);
      }
      if (checking) {
        int used = sweeps;
        for (;;) {
          run(S_RES);
          for (int m = 0; m < nr; ++m)
            HL_CHECK(launch_check_norms(mem[m].r, mem[m].b, 1.0, nullptr, 0.0, (int)N, cb.partial.as<double>(),
                                        cb.slot(m), s));
          const std::vector<double> v = cb.read(nr, s);
          double worst = 0.0;
          for (int m = 0; m < nr; ++m) {
            const double rel = rel_residual(v[2 * m], v[2 * m + 1]);
            worst = (rel > worst || std::isnan(rel)) ? rel : worst;
          }
          const bool ok = !(tol > 0.0) || worst <= tol;
          if (ok || used >= maxsw) {
            log.note(worst, used);
            if (!ok) {
              if (stats) {
                stats->steps_done = written;
                stats->seconds = now_s() - t_start;
              }
              return fail(HLEVY_ERR_NOT_CONVERGED,
                          "refinement reached a relative residual of " + std::to_string(worst) + " after " +
                              std::to_string(used) + " sweeps (tol " + std::to_string(tol) + ") in columns " +
                              std::to_string(c0) + ".." + std::to_string(c0 + nr - 1));
            }
            break;
          }
          run(S_L1);
          run(S_ADD);
          ++used;
        }
      }
      for (int m = 0; m < nr; ++m)
        HL_CHECK(launch_perm_scatter(x + (size_t)(c0 + m) * ld, mem[m].x, perm, (int)N, s));
      written += nr;
    }
    // the work vectors are freed on return: wait for the device first
    HL_CHECK(hipStreamSynchronize(s));
    if (stats) {
      stats->steps_done = written;
      stats->seconds = now_s() - t_start;
    }
    return HLEVY_OK;
  });
}

hlevy_status hlevy_solve_noalloc(hlevy_fac* f, const double* b, double* x, const hlevy_refine* refine,
                                 hlevy_stats* stats, void* stream) {
  if (!f || !b || !x) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  const int64_t N = f->op->S.N;
  if (N > HLEVY_NOALLOC_MAX_N)
    return fail(HLEVY_ERR_INVALID_ARG, "hlevy_solve_noalloc takes N <= " + std::to_string(HLEVY_NOALLOC_MAX_N) +
                                           " (its scratch size); use hlevy_solve");
  if (b < x + N && x < b + N) return fail(HLEVY_ERR_INVALID_ARG, "b and x must not overlap");
  if (const char* e = refine_error(refine)) return fail(HLEVY_ERR_INVALID_ARG, e);
  const double t_start = now_s();
  CheckLog log{stats};
  log.begin(f);
  return guarded([&]() -> hlevy_status {
    hipStream_t s = as_stream(stream);
    double* work = scratch_ptr();
    const int sweeps = default_sweeps(f, refine);
    const double tol = refine ? refine->tol : 0.0;
    const int maxsw = std::max(sweeps, refine ? refine->max_sweeps : 0);
    const hlevy_status st = solve_column(f, b, x, work, work + 4 * (size_t)N, sweeps, tol, maxsw,
                                         stats || tol > 0.0, log, s);
    if (stats) {
      stats->steps_done = st == HLEVY_OK ? 1 : 0;
      stats->seconds = now_s() - t_start;
    }
    return st;
  });
}

// Steady solves (shift I - G) x = b by conjugate gradients or BiCGSTAB, the
// factor's inverse factors as the preconditioner (Sec. 5.1, 5.3, 5.4).
// Vectors are in cluster order; the scalars of the iteration stay in a
// device array (see krylov.hip) and the host reads them once per half
// iteration for the stopping test.
hlevy_status hlevy_krylov_solve(hlevy_fac* f, const double* b, double* x, const hlevy_krylov* opt,
                                hlevy_krylov_stats* stats, double* history, void* stream) {
  if (!f || !b || !x || !opt) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  const int N = f->op->S.N;
  if (b < x + N && x < b + N) return fail(HLEVY_ERR_INVALID_ARG, "b and x must not overlap");
  if (opt->method != HLEVY_KRYLOV_CG && opt->method != HLEVY_KRYLOV_BICGSTAB && opt->method != HLEVY_KRYLOV_GMRES)
    return fail(HLEVY_ERR_INVALID_ARG, "method must be HLEVY_KRYLOV_CG, HLEVY_KRYLOV_BICGSTAB or HLEVY_KRYLOV_GMRES");
  if (opt->method == HLEVY_KRYLOV_GMRES && (opt->restart < 0 || opt->restart > 64))
    return fail(HLEVY_ERR_INVALID_ARG, "restart must lie in [0, 64]");
  if (opt->max_iter < 1) return fail(HLEVY_ERR_INVALID_ARG, "max_iter must be >= 1");
  if (!(opt->tol >= 0.0) || !std::isfinite(opt->tol)) return fail(HLEVY_ERR_INVALID_ARG, "tol must be finite and >= 0");
  if (!std::isfinite(opt->shift)) return fail(HLEVY_ERR_INVALID_ARG, "shift must be finite");
  if ((opt->precondition != 0 && opt->precondition != 1) || (opt->use_guess != 0 && opt->use_guess != 1))
    return fail(HLEVY_ERR_INVALID_ARG, "precondition and use_guess are 0 or 1");
  // the iteration's operator: the factor's own, or one with its ordering
  const hlevy_op* aop = opt->op ? opt->op : f->op;
  if (aop != f->op && (aop->S.N != N || aop->S.perm != f->op->S.perm))
    return fail(HLEVY_ERR_INVALID_ARG, "op must have the factor's points in the factor's cluster order");
  const MvPlan& mvA = aop == f->op ? f->mvG : aop->mv;
  const double t_start = now_s();
  return guarded([&]() -> hlevy_status {
    hipStream_t s = as_stream(stream);
    const int32_t* perm = f->op->ds.perm.as<int32_t>();
    enum { V_B, V_X, V_R, V_P, V_Q, V_Z, V_T, V_S, V_RH, V_W, NV };
    enum { S_ONE, S_BB, S_RR, S_RZ, S_RZOLD, S_PQ, S_ALPHA, S_BETA, S_BW, S_OMEGA, S_RHO, S_RHOOLD, S_RV, S_TS,
           S_TT, S_SS, NS = 32 };
    const size_t nd = (size_t)KR_MAXDOT * kr_blocks(N);
    DevBuf work;
    work.alloc((NV * (size_t)N + nd + NS) * sizeof(double));
    double* v[NV];
    for (int i = 0; i < NV; ++i) v[i] = work.as<double>() + (size_t)i * N;
    double* partial = work.as<double>() + NV * (size_t)N;
    double* sc = partial + nd;
    double init[NS] = {};
    init[S_ONE] = 1.0;
    HL_CHECK(hipMemcpyAsync(sc, init, sizeof(init), hipMemcpyHostToDevice, s));
    const KrCoef one{-1, 0, 1.0}, none{-1, 0, 0.0}, minus{-1, 0, -1.0};
    auto sc_coef = [](int idx, double mul) { return KrCoef{idx, 0, mul}; };
    auto comb = [&](double* out, const double* a, KrCoef ca, const double* b1 = nullptr, KrCoef cb = KrCoef{},
                    const double* c1 = nullptr, KrCoef cc = KrCoef{}) {
      HL_CHECK(launch_kr_comb(out, a, ca, b1, cb, c1, cc, sc, N, s));
    };
    struct DotReq {
      const double* a;
      const double* b;
      int out;
    };
    auto dots = [&](std::initializer_list<DotReq> l) {
      KrDots d{};
      for (const DotReq& e : l) {
        d.a[d.n] = e.a;
        d.b[d.n] = e.b;
        d.out[d.n] = e.out;
        ++d.n;
      }
      HL_CHECK(launch_kr_dots(d, N, partial, sc, s));
    };
    auto dot_to = [](const double* a, const double* b1, int out) { return DotReq{a, b1, out}; };
    auto ratios = [&](std::initializer_list<KrRatio> l) {
      KrRatios q{};
      for (const auto& r : l) q.r[q.n++] = r;
      HL_CHECK(launch_kr_scalars(q, sc, s));
    };
    double host[NS];
    auto read = [&]() {
      HL_CHECK(hipMemcpyAsync(host, sc, sizeof(host), hipMemcpyDeviceToHost, s));
      HL_CHECK(hipStreamSynchronize(s));
    };
    // A y = shift y - G y (FP64 operator)
    auto apply_A = [&](const double* y, double* out) {
      MvEpi e{};
      e.kind = MV_EPI_AXPY;
      e.hdt = -1.0;
      e.cg = opt->shift;
      e.g = y;
      e.y = out;
      mvA.run(y, e, s);
    };
    auto precond = [&](const double* y, double* out) {
      if (!opt->precondition) {
        comb(out, y, one);
        return;
      }
      f->mvLi.run(y, epi_plain(v[V_W]), s);
      f->mvUi.run(v[V_W], epi_plain(out), s);
    };
    HL_CHECK(launch_perm_gather(v[V_B], b, perm, N, s));
    if (opt->use_guess) {
      HL_CHECK(launch_perm_gather(v[V_X], x, perm, N, s));
      apply_A(v[V_X], v[V_Q]);
      comb(v[V_R], v[V_B], one, v[V_Q], minus);
    } else {
      comb(v[V_X], v[V_B], none);
      comb(v[V_R], v[V_B], one);
    }
    dots({dot_to(v[V_B], v[V_B], S_BB), dot_to(v[V_R], v[V_R], S_RR)});
    read();
    const double bnorm = std::sqrt(host[S_BB]);
    int it = 0;
    bool converged = false;
    double rel = 0.0;
    if (bnorm == 0.0) {
      comb(v[V_X], v[V_B], none);   // b = 0: x = 0
      converged = true;
    } else {
      rel = std::sqrt(host[S_RR]) / bnorm;
      if (history) history[0] = rel;
      converged = rel <= opt->tol;
      const double tol = opt->tol;
      auto check = [&](double rr) {
        rel = std::sqrt(rr) / bnorm;
        if (history) history[it] = rel;
        return std::isfinite(rel) && rel <= tol;
      };
      if (opt->method == HLEVY_KRYLOV_CG) {
        double *r = v[V_R], *p = v[V_P], *q = v[V_Q], *z = v[V_Z], *xv = v[V_X];
        precond(r, z);
        dots({dot_to(r, z, S_RZ)});
        comb(p, z, one);
        while (!converged && it < opt->max_iter && std::isfinite(rel)) {
          ++it;
          apply_A(p, q);
          dots({dot_to(p, q, S_PQ)});
          ratios({KrRatio{S_ALPHA, S_RZ, S_PQ, -1, -1, S_RZ, S_RZOLD, 0}});
          comb(xv, xv, one, p, sc_coef(S_ALPHA, 1.0));
          comb(r, r, one, q, sc_coef(S_ALPHA, -1.0));
          precond(r, z);
          dots({dot_to(r, r, S_RR), dot_to(r, z, S_RZ)});
          read();
          converged = check(host[S_RR]);
          if (converged || !std::isfinite(rel)) break;
          ratios({KrRatio{S_BETA, S_RZ, S_RZOLD, -1, -1, -1, -1, 0}});
          comb(p, z, one, p, sc_coef(S_BETA, 1.0));
        }
      } else if (opt->method == HLEVY_KRYLOV_GMRES) {
        // restarted GMRES, right-preconditioned: Arnoldi on A M^{-1} with
        // classical Gram-Schmidt applied twice (coefficients reduced on the
        // device, read back once per step with the new vector's norm), the
        // Givens rotations and the least-squares solve on the host, and
        // x += M^{-1} V y at the end of each cycle
        const int m = opt->restart > 0 ? opt->restart : 30;
        const int nbk = kr_blocks(N);
        DevBuf gw;
        gw.alloc(((size_t)(m + 1) * N + (size_t)(m + 1) * nbk + 3 * (size_t)(m + 1)) * sizeof(double));
        double* V = gw.as<double>();
        double* gpart = V + (size_t)(m + 1) * N;
        double* h1 = gpart + (size_t)(m + 1) * nbk;   // first pass coefficients, then the norm at [j + 1]
        double* h2 = h1 + (m + 1);                     // second pass
        double* yc = h2 + (m + 1);                     // the cycle's solution coefficients
        double *xv = v[V_X], *r = v[V_R], *w = v[V_Q], *z = v[V_Z], *pz = v[V_P];
        std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), hb(2 * (m + 1)), y(m);
        double beta = std::sqrt(host[S_RR]);
        while (!converged && it < opt->max_iter && std::isfinite(rel) && beta > 0.0) {
          comb(V, r, KrCoef{-1, 0, 1.0 / beta});
          std::fill(g.begin(), g.end(), 0.0);
          g[0] = beta;
          int jend = 0;
          for (int j = 0; j < m && it < opt->max_iter; ++j) {
            ++it;
            double* vj = V + (size_t)j * N;
            precond(vj, z);
            apply_A(z, w);
            HL_CHECK(launch_gm_dots(V, N, j + 1, w, N, gpart, h1, s));
            HL_CHECK(launch_gm_comb(w, w, V, N, j + 1, h1, -1.0, N, s));
            HL_CHECK(launch_gm_dots(V, N, j + 1, w, N, gpart, h2, s));
            HL_CHECK(launch_gm_comb(w, w, V, N, j + 1, h2, -1.0, N, s));
            HL_CHECK(launch_gm_dots(w, N, 1, w, N, gpart, h1 + j + 1, s));
            HL_CHECK(hipMemcpyAsync(hb.data(), h1, 2 * (m + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
            HL_CHECK(hipStreamSynchronize(s));
            double* hc = H.data() + (size_t)j * (m + 1);   // column j of the Hessenberg matrix
            for (int i = 0; i <= j; ++i) hc[i] = hb[i] + hb[(m + 1) + i];
            const double hn = std::sqrt(hb[j + 1]);
            hc[j + 1] = hn;
            jend = j + 1;
            if (hn > 0.0) comb(V + (size_t)(j + 1) * N, w, KrCoef{-1, 0, 1.0 / hn});
            for (int i = 0; i < j; ++i) {   // earlier rotations
              const double a0 = hc[i], a1 = hc[i + 1];
              hc[i] = cs[i] * a0 + sn[i] * a1;
              hc[i + 1] = -sn[i] * a0 + cs[i] * a1;
            }
            const double den = std::hypot(hc[j], hc[j + 1]);
            cs[j] = den > 0.0 ? hc[j] / den : 1.0;
            sn[j] = den > 0.0 ? hc[j + 1] / den : 0.0;
            hc[j] = den;
            hc[j + 1] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            rel = std::fabs(g[j + 1]) / bnorm;
            if (history) history[it] = rel;
            converged = std::isfinite(rel) && rel <= tol;
            if (converged || !std::isfinite(rel) || hn == 0.0) break;
          }
          // y = R^{-1} g (back substitution), x += M^{-1} V y
          for (int i = jend - 1; i >= 0; --i) {
            double acc = g[i];
            for (int k = i + 1; k < jend; ++k) acc -= H[(size_t)k * (m + 1) + i] * y[k];
            y[i] = acc / H[(size_t)i * (m + 1) + i];
          }
          HL_CHECK(hipMemcpyAsync(yc, y.data(), jend * sizeof(double), hipMemcpyHostToDevice, s));
          HL_CHECK(launch_gm_comb(w, nullptr, V, N, jend, yc, 1.0, N, s));
          precond(w, pz);
          comb(xv, xv, one, pz, one);
          if (converged || !std::isfinite(rel) || it >= opt->max_iter) break;
          // restart from the true residual
          apply_A(xv, w);
          comb(r, v[V_B], one, w, minus);
          dots({dot_to(r, r, S_RR)});
          read();
          beta = std::sqrt(host[S_RR]);
          rel = beta / bnorm;
          converged = rel <= tol;
        }
      } else {
        double *r = v[V_R], *p = v[V_P], *vv = v[V_Q], *y = v[V_Z], *t = v[V_T], *sv = v[V_S], *rh = v[V_RH],
               *xv = v[V_X];
        comb(rh, r, one);
        dots({dot_to(rh, r, S_RHO), dot_to(rh, r, S_RHOOLD)});
        while (!converged && it < opt->max_iter && std::isfinite(rel)) {
          ++it;
          if (it == 1) {
            comb(p, r, one);
          } else {
            // beta = (rho_i / rho_{i-1}) (alpha / omega); p = r + beta (p - omega v)
            ratios({KrRatio{S_BETA, S_RHO, S_RHOOLD, S_ALPHA, S_OMEGA, -1, -1, 0},
                    KrRatio{S_BW, S_RHO, S_RHOOLD, S_ALPHA, S_ONE, S_RHO, S_RHOOLD, 0}});
            comb(p, r, one, p, sc_coef(S_BETA, 1.0), vv, sc_coef(S_BW, -1.0));
          }
          precond(p, y);
          apply_A(y, vv);
          dots({dot_to(rh, vv, S_RV)});
          ratios({KrRatio{S_ALPHA, S_RHO, S_RV, -1, -1, -1, -1, 0}});
          comb(sv, r, one, vv, sc_coef(S_ALPHA, -1.0));
          comb(xv, xv, one, y, sc_coef(S_ALPHA, 1.0));
          dots({dot_to(sv, sv, S_SS)});
          read();
          if (check(host[S_SS]) || !std::isfinite(rel)) {
            converged = std::isfinite(rel);
            comb(r, sv, one);
            break;
          }
          precond(sv, y);
          apply_A(y, t);
          dots({dot_to(t, sv, S_TS), dot_to(t, t, S_TT)});
          ratios({KrRatio{S_OMEGA, S_TS, S_TT, -1, -1, -1, -1, 0}});
          comb(xv, xv, one, y, sc_coef(S_OMEGA, 1.0));
          comb(r, sv, one, t, sc_coef(S_OMEGA, -1.0));
          dots({dot_to(r, r, S_RR), dot_to(rh, r, S_RHO)});
          read();
          converged = check(host[S_RR]);
        }
      }
      // the residual of the returned x, with the FP64 operator
      apply_A(v[V_X], v[V_Q]);
      comb(v[V_T], v[V_B], one, v[V_Q], minus);
      dots({dot_to(v[V_T], v[V_T], S_RR)});
      read();
      rel = std::sqrt(host[S_RR]) / bnorm;
    }
    HL_CHECK(launch_perm_scatter(x, v[V_X], perm, N, s));
    HL_CHECK(hipStreamSynchronize(s));
    if (stats) {
      stats->iterations = it;
      stats->converged = converged ? 1 : 0;
      stats->rel_residual = rel;
      stats->seconds = now_s() - t_start;
    }
    if (!converged)
      return fail(HLEVY_ERR_NOT_CONVERGED, "Krylov iteration reached a relative residual of " + std::to_string(rel) +
                                               " after " + std::to_string(it) + " iterations (tol " +
                                               std::to_string(opt->tol) + ")");
    return HLEVY_OK;
  });
}

hlevy_status hlevy_step(hlevy_fac* f, double* u, int64_t nsteps, const double* g, const double* phi,
                        const hlevy_refine* refine, hlevy_stats* stats, void* stream) {
  if (!f || !u) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  if (nsteps < 0) return fail(HLEVY_ERR_INVALID_ARG, "nsteps must be >= 0");
  if (g && !phi) return fail(HLEVY_ERR_INVALID_ARG, "phi is required with g");
  if (const char* e = refine_error(refine)) return fail(HLEVY_ERR_INVALID_ARG, e);
  if (g)
    for (int64_t i = 0; i <= nsteps; ++i)
      if (!std::isfinite(phi[i])) return fail(HLEVY_ERR_INVALID_ARG, "non-finite phi");
  const double t_start = now_s();
  CheckLog log{stats};
  log.begin(f);
  return guarded([&]() -> hlevy_status {
    hipStream_t s = as_stream(stream);
    const int N = f->op->S.N;
    const int32_t* perm = f->op->ds.perm.as<int32_t>();
    const double hdt = 0.5 * f->dt;
    const int sweeps = default_sweeps(f, refine);
    const double tol = refine ? refine->tol : 0.0;
    const int every = refine ? refine->check_every : 0;
    const int maxsw = std::max(sweeps, refine ? refine->max_sweeps : 0);
    const bool checking = stats || tol > 0.0;
    CheckBuf cb;
    if (checking) cb.reserve(1, N);
    // Since I + dt/2 G = 2 I - M, each step solves M w = 2 u^n + F_n
    // (F_n = dt/2 (phi_n + phi_{n+1}) g) and sets u^{n+1} = w - u^n: one
    // product with G per refinement sweep and none for the right side.
    double* uc = f->w_u.as<double>();   // u^n
    double* w = f->w_d.as<double>();    // iterate of M w = 2 u^n + F_n
    double* z = f->w_z.as<double>();
    double* r = f->w_y.as<double>();
    double* gc = f->w_g.as<double>();   // g (cluster order)
    double* lg = f->w_b.as<double>();   // L^{-1} g
    HL_CHECK(launch_perm_gather(uc, u, perm, N, s));
    if (g) {
      HL_CHECK(launch_perm_gather(gc, g, perm, N, s));
      f->mvLi.run(gc, epi_plain(lg), s);
    }
    auto cn_residual = [&](double cg) {
      MvEpi e3{};
      e3.kind = MV_EPI_CNRES;   // r = 2 u^n + F_n - (w - dt/2 G w)
      e3.hdt = hdt;
      e3.cg = cg;
      e3.u = uc;
      e3.g = g ? gc : nullptr;
      e3.b = w;
      e3.y = r;
      f->mvG.run(w, e3, s);
    };
    auto add_update = [&]() {
      MvEpi e4{};
      e4.kind = MV_EPI_ADD;   // w += U^{-1} L^{-1} r
      e4.u = w;
      e4.y = w;
      f->mvLi.run(r, epi_plain(z), s);
      f->mvUi.run(z, e4, s);
    };
    for (int64_t n = 0; n < nsteps; ++n) {
      const double cg = g ? hdt * (phi[n] + phi[n + 1]) : 0.0;
      const bool chk = checking && (n + 1 == nsteps || (every > 0 && (n + 1) % every == 0));
      // z = L^{-1} (2 u^n + F_n) = 2 L^{-1} u^n + cg L^{-1} g
      MvEpi e{};
      e.kind = MV_EPI_AXPY;
      e.hdt = 2.0;
      e.cg = cg;
      e.g = g ? lg : nullptr;
      e.y = z;
      f->mvLi.run(uc, e, s);
      if (sweeps == 0 && !chk) {
        MvEpi e2{};
        e2.kind = MV_EPI_SUB;   // u^{n+1} = U^{-1} z - u^n
        e2.u = uc;
        e2.y = uc;
        f->mvUi.run(z, e2, s);
        continue;
      }
      f->mvUi.run(z, epi_plain(w), s);
      for (int it = 0; it < sweeps; ++it) {
        cn_residual(cg);
        if (it + 1 < sweeps || chk) {
          add_update();
        } else {
          f->mvLi.run(r, epi_plain(z), s);
          MvEpi e4{};
          e4.kind = MV_EPI_NEXT;   // u^{n+1} = w + U^{-1} L^{-1} r - u^n
          e4.b = w;
          e4.u = uc;
          e4.y = uc;
          f->mvUi.run(z, e4, s);
        }
      }
      if (chk) {
        // the residual of the final iterate w (one more product with G);
        // further sweeps while it misses the target
        int used = sweeps;
        double rel = 0.0;
        for (;;) {
          cn_residual(cg);
          HL_CHECK(launch_check_norms(r, uc, 2.0, g ? gc : nullptr, cg, N, cb.partial.as<double>(), cb.slot(0), s));
          const std::vector<double> v = cb.read(1, s);
          rel = rel_residual(v[0], v[1]);
          if (!(tol > 0.0) || rel <= tol || used >= maxsw) break;
          add_update();
          ++used;
        }
        log.note(rel, used);
        if (tol > 0.0 && !(rel <= tol)) {
          // step n is not applied: u keeps u^n, the last completed step
          HL_CHECK(launch_perm_scatter(u, uc, perm, N, s));
          HL_CHECK(hipStreamSynchronize(s));
          if (stats) {
            stats->steps_done = n;
            stats->seconds = now_s() - t_start;
          }
          return fail(HLEVY_ERR_NOT_CONVERGED, "step " + std::to_string(n) + ": relative residual " +
                                                   std::to_string(rel) + " after " + std::to_string(used) +
                                                   " sweeps (tol " + std::to_string(tol) + ")");
        }
        HL_CHECK(launch_wsub(uc, w, N, s));   // u^{n+1} = w - u^n
      }
    }
    HL_CHECK(launch_perm_scatter(u, uc, perm, N, s));
    if (stats) {
      HL_CHECK(hipStreamSynchronize(s));
      stats->steps_done = nsteps;
      stats->seconds = now_s() - t_start;
    }
    return HLEVY_OK;
  });
}

hlevy_status hlevy_step_batched(hlevy_fac* const* facs, double* const* u, const int64_t* nsteps, int32_t count,
                                const hlevy_refine* refine, hlevy_stats* stats, void* stream) {
  if (!facs || !u || !nsteps) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  if (count < 1) return fail(HLEVY_ERR_INVALID_ARG, "count must be >= 1");
  if (const char* e = refine_error(refine)) return fail(HLEVY_ERR_INVALID_ARG, e);
  int64_t nmax = 0, total = 0;
  {
    std::set<const hlevy_fac*> seen;
    for (int32_t i = 0; i < count; ++i) {
      if (!facs[i] || !u[i]) return fail(HLEVY_ERR_INVALID_ARG, "null factor or vector");
      if (nsteps[i] < 0) return fail(HLEVY_ERR_INVALID_ARG, "nsteps must be >= 0");
      if (!seen.insert(facs[i]).second) return fail(HLEVY_ERR_INVALID_ARG, "a factor appears twice in the batch");
      nmax = std::max(nmax, nsteps[i]);
      total += nsteps[i];
    }
  }
  const double t_start = now_s();
  CheckLog log{stats};
  log.begin(facs[0]);
  if (stats) {
    stats->rank_overflows = 0;
    for (int32_t i = 0; i < count; ++i) stats->rank_overflows = std::max(stats->rank_overflows, facs[i]->rank_overflows);
  }
  return guarded([&]() -> hlevy_status {
    hipStream_t s = as_stream(stream);
    int sweeps = 0;
    for (int32_t i = 0; i < count; ++i) sweeps = std::max(sweeps, default_sweeps(facs[i], refine));
    const double tol = refine ? refine->tol : 0.0;
    const bool checking = stats || tol > 0.0;
    std::vector<double> rel(count, -1.0);
    std::vector<StepState> st;
    for (int32_t i = 0; i < count; ++i) {
      hlevy_fac* f = facs[i];
      StepState x{f, f->w_u.as<double>(), f->w_d.as<double>(), f->w_z.as<double>(), f->w_y.as<double>(),
                  nullptr, nullptr, nullptr, nsteps[i]};
      x.check = checking && nsteps[i] > 0;
      x.rel = &rel[i];
      st.push_back(x);
      HL_CHECK(launch_perm_gather(st.back().uc, u[i], f->op->ds.perm.as<int32_t>(), f->op->S.N, s));
    }
    step_states(st, nmax, sweeps, s);
    for (int32_t i = 0; i < count; ++i)
      HL_CHECK(launch_perm_scatter(u[i], st[i].uc, facs[i]->op->ds.perm.as<int32_t>(), facs[i]->op->S.N, s));
    HL_CHECK(hipStreamSynchronize(s));
    int worst = -1;
    for (int32_t i = 0; i < count; ++i) {
      if (rel[i] < 0.0 && !std::isnan(rel[i])) continue;
      log.note(rel[i], sweeps);
      if (worst < 0 || !(rel[worst] >= rel[i])) worst = i;
    }
    if (stats) {
      if (worst >= 0) stats->last_rel_residual = rel[worst];
      stats->steps_done = total;
      stats->seconds = now_s() - t_start;
    }
    if (tol > 0.0 && worst >= 0 && !(rel[worst] <= tol))
      return fail(HLEVY_ERR_NOT_CONVERGED, "problem " + std::to_string(worst) + ": relative residual " +
                                               std::to_string(rel[worst]) + " of its last step (tol " +
                                               std::to_string(tol) + ")");
    return HLEVY_OK;
  });
}

hlevy_status hlevy_fac_apply(hlevy_fac* f, int32_t which, const double* x, double* y, void* stream) {
  if (!f || !x || !y) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  if (x == y) return fail(HLEVY_ERR_INVALID_ARG, "x and y must not alias");
  if (which < 0 || which > 2) return fail(HLEVY_ERR_INVALID_ARG, "which must be 0, 1 or 2");
  return guarded([&]() -> hlevy_status {
    hipStream_t s = as_stream(stream);
    const int N = f->op->S.N;
    const int32_t* perm = f->op->ds.perm.as<int32_t>();
    const MvPlan& M = which == 0 ? f->mvG : (which == 1 ? f->mvLi : f->mvUi);
    HL_CHECK(launch_perm_gather(f->w_z.as<double>(), x, perm, N, s));
    M.run(f->w_z.as<double>(), epi_plain(f->w_y.as<double>()), s);
    HL_CHECK(launch_perm_scatter(y, f->w_y.as<double>(), perm, N, s));
    return HLEVY_OK;
  });
}

hlevy_status hlevy_fac_kernel_times(hlevy_fac* f, int32_t reps, void* stream, hlevy_kernel_times* out) {
  if (!f || !out) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  if (reps < 1 || reps > 100000) return fail(HLEVY_ERR_INVALID_ARG, "reps must be in [1, 100000]");
  return guarded([&]() -> hlevy_status {
    hipStream_t s = as_stream(stream);
    const MvPlan* plans[3] = {&f->mvG, &f->mvLi, &f->mvUi};
    const double* x = f->w_u.as<double>();
    double* y = f->w_y.as<double>();
    std::vector<hipEvent_t> ev((size_t)reps * 12);
    for (auto& e : ev) HL_CHECK(hipEventCreate(&e));
    const MvEpi e = epi_plain(y);
    // the products in the order of a Crank-Nicolson step (G, L^{-1}, U^{-1}),
    // so the three matrices stream through the caches as they do when
    // stepping; each kernel carries its own start/stop events
    for (int r = 0; r < reps; ++r)
      for (int w = 0; w < 3; ++w) {
        hipEvent_t* E = &ev[((size_t)r * 3 + w) * 4];
        HL_CHECK(project_launch(plans[w]->dev, x, s, E[0], E[1]));
        HL_CHECK(gather_launch(plans[w]->dev, x, e, s, E[2], E[3]));
      }
    HL_CHECK(hipStreamSynchronize(s));
    std::memset(out, 0, sizeof(*out));
    for (int r = 0; r < reps; ++r)
      for (int w = 0; w < 3; ++w) {
        hipEvent_t* E = &ev[((size_t)r * 3 + w) * 4];
        float a = 0.f, b = 0.f;
        if (plans[w]->dev.ntiles > 0) HL_CHECK(hipEventElapsedTime(&a, E[0], E[1]));
        HL_CHECK(hipEventElapsedTime(&b, E[2], E[3]));
        out->project_ms[w] += a / reps;
        out->gather_ms[w] += b / reps;
      }
    for (auto& e : ev) (void)hipEventDestroy(e);
    for (int w = 0; w < 3; ++w) {
      const MvPlan& M = *plans[w];
      out->dense_bytes[w] = (double)M.dense_bytes;
      out->u_bytes[w] = (double)M.u_bytes;
      out->v_bytes[w] = (double)M.v_bytes;
      out->partial_bytes[w] = (double)M.nslots * M.dev.kb * sizeof(double);
    }
    out->N = f->op->S.N;
    out->reps = reps;
    return HLEVY_OK;
  });
}

void hlevy_op_destroy(hlevy_op* op) { delete op; }
void hlevy_fac_destroy(hlevy_fac* f) { delete f; }

}  // extern "C"

// ---------------------------------------------------------------------------
// serving loop: requests (problem, dt, horizon, u0) arrive at any time; each
// scheduling round admits queued requests in arrival order while the memory
// of cached operators, factors and request state fits the budget (evicting
// unused cached operators, least recently used first), assembles and
// factors the operators not in the cache in one joint plan, and advances
// every active request by one chunk of steps in one batched step.
// Requests with equal operator parameters share one cached factor; each
// request has its own vectors and projection partial buffers.
// ---------------------------------------------------------------------------
namespace hl {

struct SrvEntry {
  std::unique_ptr<hlevy_op, void (*)(hlevy_op*)> op{nullptr, hlevy_op_destroy};
  std::unique_ptr<hlevy_fac, void (*)(hlevy_fac*)> fac{nullptr, hlevy_fac_destroy};
  hlevy_problem prob{};
  hlevy_hparams hp{};
  double dt = 0;
  size_t bytes = 0;
  int refs = 0;
  uint64_t last_use = 0;
};

struct SrvReq {
  int64_t id = 0;
  std::string key;
  SrvEntry* e = nullptr;
  int64_t nsteps = 0, done = 0;
  int N = 0;
  double rel = -1.0;           // relative residual of the last step
  double* out = nullptr;
  DevBuf u0;                   // staged initial condition (natural order)
  DevBuf vec, pG, pL, pU;      // state while active
  size_t bytes = 0;
};

static std::string srv_key(const hlevy_problem& p, const hlevy_hparams& hp, double dt) {
  std::string k;
  auto put = [&](const void* v, size_t n) { k.append(reinterpret_cast<const char*>(v), n); };
  put(&p.dim, 4);
  put(&p.n, 4);
  for (double v : {p.lo, p.hi, p.a, p.b[0], p.dim == 2 ? p.b[1] : 0.0, p.c, p.s, p.lambda, p.C, p.r0, p.eps2,
                   p.lambda_neg})
    put(&v, 8);
  put(&p.kernel, 4);
  put(&hp.leaf, 4);
  put(&hp.eta, 8);
  put(&hp.n_block, 4);
  put(&hp.aca_tol, 8);
  put(&hp.max_rank, 4);
  put(&hp.gather_waves, 4);
  put(&hp.rank_bucket, 4);
  put(&hp.strict_rank_cap, 4);
  put(&hp.taylor_rank, 4);
  put(&dt, 8);
  return k;
}

}  // namespace hl

struct hlevy_server {
  hlevy_server_config cfg{};
  hipStream_t s = nullptr;
  int64_t next_id = 1;
  uint64_t tick = 0;
  size_t used = 0;
  std::map<std::string, std::unique_ptr<SrvEntry>> cache;
  std::deque<std::unique_ptr<SrvReq>> queue;
  std::vector<std::unique_ptr<SrvReq>> active;
  std::deque<int64_t> finished, failed;
  hlevy_server_stats st{};
  // a round ran out of device memory building new operators: no new
  // operator is admitted until a resident one falls idle
  bool fresh_wait = false;
};

extern "C" {

hlevy_status hlevy_server_create(const hlevy_server_config* cfg, void* stream, hlevy_server** out) {
  if (!cfg || !out) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  if (cfg->prec != HLEVY_PREC_FP64 && cfg->prec != HLEVY_PREC_MIXED && cfg->prec != HLEVY_PREC_MIXED_BF16)
    return fail(HLEVY_ERR_INVALID_ARG, "bad precision");
  if (!(cfg->lu_tol > 0.0 && cfg->lu_tol < 1.0)) return fail(HLEVY_ERR_INVALID_ARG, "lu_tol must be in (0, 1)");
  if (cfg->sweeps < 0 || cfg->sweeps > 64) return fail(HLEVY_ERR_INVALID_ARG, "sweeps in [0, 64]");
  if (cfg->chunk < 1 || cfg->max_active < 1) return fail(HLEVY_ERR_INVALID_ARG, "chunk and max_active must be >= 1");
  if (std::isnan(cfg->tol) || std::isinf(cfg->tol)) return fail(HLEVY_ERR_INVALID_ARG, "tol must be finite");
  return guarded([&]() -> hlevy_status {
    auto v = std::make_unique<hlevy_server>();
    v->cfg = *cfg;
    v->st.max_rel_residual = -1.0;
    if (v->cfg.hbm_budget == 0) v->cfg.hbm_budget = (size_t)64 << 30;
    v->s = as_stream(stream);
    *out = v.release();
    return HLEVY_OK;
  });
}

hlevy_status hlevy_server_submit(hlevy_server* v, const hlevy_problem* prob, const hlevy_hparams* hp, double dt,
                                 int64_t nsteps, const double* u0, double* u_out, int64_t* id) {
  if (!v || !prob || !hp || !u0 || !u_out || !id) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(HLEVY_ERR_INVALID_ARG, "dt must be > 0");
  if (nsteps < 0) return fail(HLEVY_ERR_INVALID_ARG, "nsteps must be >= 0");
  if (prob->mask || prob->s_field)
    return fail(HLEVY_ERR_INVALID_ARG, "the server takes box problems (no mask, no s_field)");
  return guarded([&]() -> hlevy_status {
    Structure S;
    std::string e = build_structure(*prob, *hp, S);
    if (!e.empty()) return fail(HLEVY_ERR_INVALID_ARG, e);
    auto r = std::make_unique<SrvReq>();
    r->id = v->next_id++;
    r->key = srv_key(*prob, *hp, dt);
    r->nsteps = nsteps;
    r->N = S.N;
    r->out = u_out;
    r->u0.alloc((size_t)S.N * sizeof(double));
    HL_CHECK(hipMemcpyAsync(r->u0.p, u0, (size_t)S.N * sizeof(double), hipMemcpyDeviceToDevice, v->s));
    auto it = v->cache.find(r->key);
    if (it == v->cache.end()) {
      auto en = std::make_unique<SrvEntry>();
      en->prob = *prob;
      en->hp = *hp;
      en->dt = dt;
      en->bytes = footprint_bytes(S, hp->max_rank, v->cfg.prec);
      // not resident until admitted; kept so that later requests find it
      v->cache.emplace(r->key, std::move(en));
    }
    *id = r->id;
    v->queue.push_back(std::move(r));
    v->st.submitted++;
    v->st.queued = (int64_t)v->queue.size();
    return HLEVY_OK;
  });
}

hlevy_status hlevy_server_poll(hlevy_server* v, int64_t* done_ids, int32_t cap, int32_t* ndone) {
  if (!v || !ndone || (cap > 0 && !done_ids) || cap < 0) return fail(HLEVY_ERR_INVALID_ARG, "bad argument");
  return guarded([&]() -> hlevy_status {
    hipStream_t s = v->s;
    // 1. admission (arrival order) under the memory budget
    std::vector<SrvEntry*> fresh;
    while (!v->queue.empty() && (int)v->active.size() < v->cfg.max_active) {
      SrvReq* r = v->queue.front().get();
      SrvEntry* e = v->cache.at(r->key).get();
      const size_t req_bytes = (size_t)r->N * 8 * 4 + 65536;
      const bool pending_fresh = std::find(fresh.begin(), fresh.end(), e) != fresh.end();
      if (!e->op && !pending_fresh && v->fresh_wait && !v->active.empty()) {
        bool idle_op = false;
        for (auto& kv : v->cache)
          if (kv.second->op && kv.second->refs == 0) idle_op = true;
        if (!idle_op) break;   // wait for an operator to fall idle
        v->fresh_wait = false;
      }
      const size_t need = req_bytes + ((e->op || pending_fresh) ? 0 : e->bytes);
      while (v->used + need > v->cfg.hbm_budget) {
        // evict the least recently used idle resident operator (not the
        // request's own)
        SrvEntry* lru = nullptr;
        for (auto& kv : v->cache) {
          SrvEntry* c = kv.second.get();
          if (c != e && c->op && c->refs == 0 && (!lru || c->last_use < lru->last_use)) lru = c;
        }
        if (!lru) break;
        lru->fac.reset();
        lru->op.reset();
        v->used -= lru->bytes;
        v->st.evictions++;
      }
      const bool idle = v->active.empty() && fresh.empty();
      if (v->used + need > v->cfg.hbm_budget && !idle) break;   // wait for memory
      if (e->op || pending_fresh) {
        v->st.cache_hits++;
      } else {
        v->st.cache_misses++;
        fresh.push_back(e);
      }
      v->used += need;
      e->refs++;
      r->e = e;
      r->bytes = req_bytes;
      v->active.push_back(std::move(v->queue.front()));
      v->queue.pop_front();
    }
    // 2. operators not in the cache: assembly, then one joint factorisation
    if (!fresh.empty()) {
      const double t0 = now_s();
      double t1 = t0;
      hlevy_status st = HLEVY_OK;
      {
        std::vector<hlevy_problem> pr;
        std::vector<hlevy_hparams> hv;
        for (SrvEntry* e : fresh) {
          pr.push_back(e->prob);
          hv.push_back(e->hp);
        }
        std::vector<hlevy_op*> oo(fresh.size(), nullptr);
        st = hlevy_assemble_batched(pr.data(), hv.data(), (int32_t)pr.size(), nullptr, s, oo.data());
        if (st == HLEVY_OK)
          for (size_t q = 0; q < fresh.size(); ++q) fresh[q]->op.reset(oo[q]);
      }
      if (st == HLEVY_OK) {
        t1 = now_s();
        std::vector<const hlevy_op*> ops;
        std::vector<double> dts;
        for (SrvEntry* e : fresh) {
          ops.push_back(e->op.get());
          dts.push_back(e->dt);
        }
        // the joint factorisation's transient workspace comes on top of the
        // resident bytes: the arena takes half of what the device has free
        // beyond the new factors' own storage and an 8 GiB margin (the
        // product workspace grows beside it), at most the default budget
        auto workspace = [&]() -> size_t {
          size_t free_b = 0, total_b = 0;
          if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
          }
          // the margin covers what the runtime allocates beside the library
          // (the callers' tensors, kernel scratch, the plan's arrays)
          size_t need = (size_t)8 << 30;
          for (SrvEntry* e : fresh) need += e->bytes;
          const size_t floor_b = (size_t)1 << 30;
          return free_b > need + 2 * floor_b ? std::min(kDefaultFactorWorkspace, (free_b - need) / 2) : floor_b;
        };
        std::vector<hlevy_fac*> fo(fresh.size(), nullptr);
        st = hlevy_factor_batched(ops.data(), dts.data(), (int32_t)ops.size(), v->cfg.prec, v->cfg.lu_tol,
                                  workspace(), s, fo.data());
        if (st == HLEVY_ERR_OOM) {
          // the device ran out before the budget did (allocator caches and
          // fragmentation are not in the count): every idle resident
          // operator leaves and the factorisation runs once more
          HL_CHECK(hipStreamSynchronize(s));
          for (auto& kv : v->cache) {
            SrvEntry* c = kv.second.get();
            if (c->op && c->refs == 0 && std::find(fresh.begin(), fresh.end(), c) == fresh.end()) {
              c->fac.reset();
              c->op.reset();
              v->used -= c->bytes;
              v->st.evictions++;
            }
          }
          st = hlevy_factor_batched(ops.data(), dts.data(), (int32_t)ops.size(), v->cfg.prec, v->cfg.lu_tol,
                                    workspace(), s, fo.data());
        }
        if (st == HLEVY_OK)
          for (size_t q = 0; q < fresh.size(); ++q) {
            fresh[q]->fac.reset(fo[q]);
            // admission counted the estimate at rank capacity; from now on
            // the entry holds what was actually allocated
            const size_t actual = fresh[q]->op->bytes + fresh[q]->fac->bytes;
            v->used = v->used - fresh[q]->bytes + actual;
            fresh[q]->bytes = actual;
          }
      }
      if (st != HLEVY_OK) {
        // the new operators could not be built.  Out of device memory while
        // other requests hold theirs: the new requests go back to the head
        // of the queue, in order, and wait until an operator falls idle.
        // Otherwise they leave the server as failed
        // (hlevy_server_take_failed).  Either way their memory is returned,
        // the entries stay non-resident and the other active requests are
        // untouched
        const std::string msg = g_last_error;
        bool others = false;
        for (auto& r : v->active)
          if (std::find(fresh.begin(), fresh.end(), r->e) == fresh.end()) others = true;
        const bool requeue = st == HLEVY_ERR_OOM && others;
        std::vector<std::unique_ptr<SrvReq>> keep, back;
        std::string ids;
        for (auto& r : v->active) {
          if (std::find(fresh.begin(), fresh.end(), r->e) == fresh.end()) {
            keep.push_back(std::move(r));
            continue;
          }
          r->e->refs--;
          v->used -= r->bytes;
          if (requeue) {
            r->e = nullptr;
            r->bytes = 0;
            back.push_back(std::move(r));
            continue;
          }
          v->failed.push_back(r->id);
          v->st.failed++;
          ids += (ids.empty() ? "" : ",") + std::to_string(r->id);
        }
        v->active.swap(keep);
        for (SrvEntry* e : fresh) {
          e->fac.reset();
          e->op.reset();
          v->used -= e->bytes;
        }
        if (requeue) {
          // admission counted one miss per new operator and a hit for each
          // further request of it; they are counted again when readmitted
          v->st.cache_misses -= (int64_t)fresh.size();
          v->st.cache_hits -= (int64_t)(back.size() - fresh.size());
          for (auto it = back.rbegin(); it != back.rend(); ++it) v->queue.push_front(std::move(*it));
          v->fresh_wait = true;
        }
        v->st.active = (int64_t)v->active.size();
        v->st.queued = (int64_t)v->queue.size();
        if (!requeue) {
          *ndone = 0;
          return fail(st, msg + " (requests " + ids + " failed)");
        }
      } else {
        v->st.assemble_seconds += t1 - t0;
        v->st.factor_seconds += now_s() - t1;
      }
    }
    // 3. state of newly active requests
    for (auto& r : v->active) {
      if (r->vec.p) continue;
      hlevy_fac* f = r->e->fac.get();
      r->vec.alloc((size_t)r->N * 4 * sizeof(double));
      r->pG.alloc(std::max<int64_t>(f->mvG.nslots, 1) * f->mvG.dev.kb * sizeof(double));
      r->pL.alloc(std::max<int64_t>(f->mvLi.nslots, 1) * f->mvLi.dev.kb * sizeof(double));
      r->pU.alloc(std::max<int64_t>(f->mvUi.nslots, 1) * f->mvUi.dev.kb * sizeof(double));
      HL_CHECK(launch_perm_gather(r->vec.as<double>(), r->u0.as<double>(), f->op->ds.perm.as<int32_t>(), r->N, s));
      r->u0.reset();
    }
    // 4. one chunk of steps for every active request
    if (!v->active.empty()) {
      // each request takes min(chunk, steps left) steps of the round
      std::vector<StepState> sts;
      int64_t c = 0, total = 0;
      for (auto& r : v->active) {
        const int64_t k = std::min<int64_t>(v->cfg.chunk, r->nsteps - r->done);
        if (k <= 0) continue;
        double* b = r->vec.as<double>();
        sts.push_back(StepState{r->e->fac.get(), b, b + r->N, b + 2 * (size_t)r->N, b + 3 * (size_t)r->N,
                                r->pG.as<double>(), r->pL.as<double>(), r->pU.as<double>(), k});
        // a request's last step measures its residual
        sts.back().check = r->done + k == r->nsteps;
        sts.back().rel = &r->rel;
        c = std::max(c, k);
        total += k;
      }
      if (c > 0) {
        const double t0 = now_s();
        step_states(sts, c, v->cfg.sweeps, s);
        v->st.step_seconds += now_s() - t0;
        for (auto& r : v->active) r->done += std::min<int64_t>(v->cfg.chunk, r->nsteps - r->done);
        v->st.problem_steps += total;
      }
    }
    // 5. finished requests: result to the caller's vector, state released
    ++v->tick;
    std::vector<std::unique_ptr<SrvReq>> keep;
    for (auto& r : v->active) {
      if (r->done < r->nsteps) {
        keep.push_back(std::move(r));
        continue;
      }
      HL_CHECK(launch_perm_scatter(r->out, r->vec.as<double>(), r->e->fac->op->ds.perm.as<int32_t>(), r->N, s));
      HL_CHECK(hipStreamSynchronize(s));
      r->e->refs--;
      r->e->last_use = v->tick;
      v->used -= r->bytes;
      v->finished.push_back(r->id);
      v->st.completed++;
      if (r->rel >= 0.0 || std::isnan(r->rel)) {
        if (!(v->st.max_rel_residual >= r->rel)) v->st.max_rel_residual = r->rel;
        if (v->cfg.tol > 0.0 && !(r->rel <= v->cfg.tol)) v->st.not_converged++;
      }
    }
    v->active.swap(keep);
    HL_CHECK(hipStreamSynchronize(s));
    int32_t n = 0;
    while (n < cap && !v->finished.empty()) {
      done_ids[n++] = v->finished.front();
      v->finished.pop_front();
    }
    *ndone = n;
    v->st.active = (int64_t)v->active.size();
    v->st.queued = (int64_t)v->queue.size();
    return HLEVY_OK;
  });
}

hlevy_status hlevy_server_take_failed(hlevy_server* v, int64_t* ids, int32_t cap, int32_t* n) {
  if (!v || !n || cap < 0 || (cap > 0 && !ids)) return fail(HLEVY_ERR_INVALID_ARG, "bad argument");
  int32_t k = 0;
  while (k < cap && !v->failed.empty()) {
    ids[k++] = v->failed.front();
    v->failed.pop_front();
  }
  *n = k;
  return HLEVY_OK;
}

hlevy_status hlevy_server_stats_get(hlevy_server* v, hlevy_server_stats* out) {
  if (!v || !out) return fail(HLEVY_ERR_INVALID_ARG, "null argument");
  *out = v->st;
  int64_t res = 0;
  for (auto& kv : v->cache) res += kv.second->op ? 1 : 0;
  out->cached_operators = res;
  out->bytes_in_use = v->used;
  return HLEVY_OK;
}

void hlevy_server_destroy(hlevy_server* v) {
  if (!v) return;
  (void)hipStreamSynchronize(v->s);
  delete v;
}

}  // extern "C"
