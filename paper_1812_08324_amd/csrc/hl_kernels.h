// Launchers of the HIP kernels (defined in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "hl_jobs.h"

namespace hl {

hipError_t launch_constants(const ProblemDev& P, double* out, hipStream_t s);
// variable-order kernel: 5 constants per distinct jump index (P.nvar blocks)
hipError_t launch_constants_var(const ProblemDev& P, double* out, hipStream_t s);
hipError_t launch_fill_dense(const ProblemDev& P, const double* cst, const int32_t* perm,
                             const LeafDesc* L, const int32_t* ids, int n, hipStream_t s);
hipError_t launch_aca(const ProblemDev& P, const int32_t* perm, const LeafDesc* L, const int32_t* ids,
                      int n, double* U, double* V, const int64_t* uoff, const int64_t* voff,
                      int32_t* ranks, int kcap, double eps, hipStream_t s);
// Forcing of a non-zero exterior (1D): tab holds 2 (n + 1) + 1 doubles of
// workspace, g is written in natural order (length n)
hipError_t launch_exterior(const ProblemDev& P, const double* cst, const double* u_ext, double* tab, double* g,
                           hipStream_t s);
// Fixed-rank Taylor factors of the Gaussian kernel straight into the
// admissible leaves ids[0..n) (rank set to r)
// 2D exterior forcing (u_ext: lattice index a at a + org per axis, ld per
// row); tab holds (2 n + 3)^2 doubles
hipError_t launch_exterior2(const ProblemDev& P, const double* cst, const double* u_ext, int ld, int org,
                            double* tab, double* g, hipStream_t s);
// g += 2D far field; tab holds (2 next + 1)^2 + 2 doubles
hipError_t launch_far_field2(const ProblemDev& P, const double* u_ext, int next, double tail_left,
                             double tail_right, double* tab, double* g, hipStream_t s);
// g += far field of an exterior on an extended lattice (1D); tab holds
// 2 (next - n) + 2 doubles
hipError_t launch_far_field(const ProblemDev& P, const double* u_ext, int next, double tail_left,
                            double tail_right, double* tab, double* g, hipStream_t s);
hipError_t launch_taylor(const ProblemDev& P, const int32_t* perm, const LeafDesc* L, const int32_t* ids, int n,
                         int32_t* rank, int r, hipStream_t s);
hipError_t launch_flush_lr(const LFlushTarget* tg, int ntg, const Term* terms, const ChunkItem* gram,
                           int ngram, const ChunkItem* expand, int nexp, double tol, int ks, hipStream_t s);
hipError_t launch_flush_dense(const DFlushItem* items, int n, const Term* terms, hipStream_t s);
hipError_t launch_dense_prod(const DProdItem* items, int n, hipStream_t s);
hipError_t launch_copy(const CopyItem* items, int n, hipStream_t s);
hipError_t launch_getrf_inv(const GetrfItem* items, int n, int32_t* zero_pivot, hipStream_t s);
// whole rounded additions (targets of at most GRAM_CHUNK rows per side, ks <= 48)
// the fused rounded additions of tg and, in the same launch, the dense
// flushes dflush (independent leaves of the same batch)
hipError_t launch_radd_fused(const LFlushTarget* tg, int ntg, const Term* terms, double tol, int ks, hipStream_t s,
                             const DFlushItem* dflush = nullptr, int ndflush = 0, const Term* dterms = nullptr);
hipError_t launch_lu_inv(const LuInvItem* items, int n, int32_t* zero_pivot, hipStream_t s);
hipError_t launch_apply(const ApplyJob* jobs, const ProjItem* proj, int nproj, const GatherItem* gat,
                        int ngat, hipStream_t s);
hipError_t launch_perm_gather(double* out, const double* in, const int32_t* perm, int N, hipStream_t s);
hipError_t launch_perm_scatter(double* out, const double* in, const int32_t* perm, int N, hipStream_t s);
hipError_t launch_axpy2(double* out, const double* x, double a, const double* y, double cg,
                        const double* g, int N, hipStream_t s);
hipError_t launch_residual(double* r, const double* b, const double* x, const double* Gx, double hdt,
                           int N, hipStream_t s);
hipError_t launch_add(double* x, const double* d, int N, hipStream_t s);
hipError_t launch_sumsq(const double* x, int N, double* partial, int nblocks, double* out, hipStream_t s);
// Refinement check: out[0] = ||r||^2, out[1] = ||alpha u + cg g||^2 (g may be
// null); partial holds 2 * check_blocks(N) doubles.  Deterministic.
int check_blocks(int N);
hipError_t launch_check_norms(const double* r, const double* u, double alpha, const double* g, double cg, int N,
                              double* partial, double* out, hipStream_t s);
// u = w - u
hipError_t launch_wsub(double* u, const double* w, int N, hipStream_t s);
hipError_t launch_densify(const LeafDesc* L, const int32_t* rank, int nleaves, const int32_t* perm,
                          int N, double* dense, hipStream_t s);
hipError_t init_kernel_attributes();

// Krylov iterations (krylov.hip).  Scalars live in a device array sc.
// A coefficient is mul * sc[idx] (idx >= 0) or the constant mul (idx < 0).
struct KrCoef {
  int32_t idx;
  int32_t pad;
  double mul;
};
constexpr int KR_MAXDOT = 3;
// up to KR_MAXDOT dot products a_k . b_k, written to sc[out[k]]
struct KrDots {
  const double* a[KR_MAXDOT];
  const double* b[KR_MAXDOT];
  int32_t out[KR_MAXDOT];
  int32_t n;
};
// sc[dst] = sc[num] / sc[den] (times sc[num2] / sc[den2] when num2 >= 0);
// after that, sc[copy_to] = sc[copy_from] when copy_from >= 0
struct KrRatio {
  int32_t dst, num, den, num2, den2, copy_from, copy_to, pad;
};
constexpr int KR_MAXRATIO = 4;
struct KrRatios {
  KrRatio r[KR_MAXRATIO];
  int32_t n, pad;
};
// partial holds KR_MAXDOT * kr_blocks(N) doubles
// GMRES: out[c] = (V column c, w) for c < ncol (fixed-order reduction;
// partial holds ncol * kr_blocks(N) doubles), and out = base + sign V coef
hipError_t launch_gm_dots(const double* V, int ld, int ncol, const double* w, int N, double* partial, double* out,
                          hipStream_t s);
hipError_t launch_gm_comb(double* out, const double* base, const double* V, int ld, int ncol, const double* coef,
                          double sign, int N, hipStream_t s);
int kr_blocks(int N);
hipError_t launch_kr_dots(const KrDots& d, int N, double* partial, double* sc, hipStream_t s);
hipError_t launch_kr_scalars(const KrRatios& q, double* sc, hipStream_t s);
// out = c0 x0 + c1 x1 + c2 x2 (x1, x2 may be null)
hipError_t launch_kr_comb(double* out, const double* x0, KrCoef c0, const double* x1, KrCoef c1,
                          const double* x2, KrCoef c2, const double* sc, int N, hipStream_t s);

inline int npairs_host(int K) { return K * (K + 1) / 2; }

}  // namespace hl
