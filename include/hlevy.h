/*
 * hlevy.h -- C ABI of the MI355X (gfx950) H-matrix Crank-Nicolson solver for
 * convection-diffusion equations driven by a Levy process.
 *
 * Method: Xu & Darve, "Efficient Numerical Method for Models Driven by Levy
 * Process via Hierarchical Matrices" (arXiv 1812.08324).
 *
 *   u_t = a Lap u + b . grad u + c u + L u          (Sec. 3.1, eq. equ:ut)
 *   L u = int (u(x+y) - u(x) - rho(y) grad u(x).y) nu(y) dy,
 *   nu(y) = C exp(-lambda |y|) / |y|^{d+2s}          (Sec. 4, eq. equ:ny2)
 *
 * discretised on a uniform grid of a box with zero exterior, the jump part by
 * singularity subtraction (Sec. 4, eqs. equ:I1approx - equ:I3approx), stored
 * as an H-matrix (App. B.1) and advanced with Crank-Nicolson (Sec. 3.2,
 * eq. equ:scheme):  (I - dt/2 G) u^{n+1} = (I + dt/2 G) u^n + dt/2 (f^n + f^{n+1}).
 *
 * Conventions shared by every entry point
 *  - Vectors are device pointers to double, length N, in natural order
 *    (1D: x_i = lo + (i+1) h; 2D: index p*n + q for the point
 *    (lo + (p+1) h, lo + (q+1) h)).  The caller owns them.
 *  - `stream` is a hipStream_t (NULL = default stream).  Work is enqueued on
 *    it; calls return before the device work finishes unless stated.
 *  - Every call returns an hlevy_status; on error the outputs are unchanged
 *    (hlevy_step: u holds the last completed step) and hlevy_last_error()
 *    describes the failure.  No C++ exception crosses this boundary.
 *  - Handles are not thread safe; distinct handles are independent.
 *  - The library allocates its device memory itself (hipMalloc) and frees it
 *    in the *_destroy calls.
 */
#ifndef HLEVY_H
#define HLEVY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HLEVY_ABI_VERSION 6

typedef enum {
  HLEVY_OK = 0,
  HLEVY_ERR_INVALID_ARG = -1,   /* bad descriptor, size or pointer */
  HLEVY_ERR_OOM = -2,           /* device allocation failed */
  HLEVY_ERR_DEVICE = -3,        /* HIP runtime error (no device, launch failure) */
  HLEVY_ERR_NOT_CONVERGED = -4, /* refinement did not reach its tolerance */
  HLEVY_ERR_RANK_CAP = -5,      /* a low-rank block needed more than its rank capacity */
  HLEVY_ERR_BAD_HANDLE = -6,
  HLEVY_ERR_ZERO_PIVOT = -7     /* a diagonal leaf had a zero pivot in the H-LU */
} hlevy_status;

typedef enum {
  HLEVY_PREC_FP64 = 0,        /* FP64 factors, plain forward/backward solve */
  HLEVY_PREC_MIXED = 1,       /* FP32 inverse factors as a preconditioner + FP64 iterative refinement */
  HLEVY_PREC_MIXED_BF16 = 2   /* as MIXED with the low-rank leaves of the inverse factors in BF16
                                 (dense leaves FP32, every product accumulating in FP64) */
} hlevy_precision;

/* Jump kernels.  TEMPERED: nu(y) = C exp(-lambda |y|) / |y|^{d+2s} (Sec. 4
 * eq. equ:ny2; lambda = 0 with C = c_{d,s} is the fractional Laplacian),
 * discretised with the singularity subtraction of Sec. 4.  GAUSSIAN: the
 * Merton jump density nu(y) = C exp(-eps2 |y|^2) (Sec. 3.3), bounded, so
 * discretised by the plain trapezoid rule of Sec. 3.2 (eqs. equ:dl and
 * equ:Aij): off-diagonal entries h^d nu(x_j - x_i), diagonal
 * -h^d sum over the lattice without 0 of nu(kh) (u = 0 outside the box). */
typedef enum {
  HLEVY_KERNEL_TEMPERED = 0,
  HLEVY_KERNEL_GAUSSIAN = 1,
  HLEVY_KERNEL_TEMPERED_ASYM = 2,
  HLEVY_KERNEL_VARIABLE_ORDER = 3
} hlevy_kernel;
/* TEMPERED_ASYM: the tempered kernel with rate lambda for jumps y > 0 and
 * lambda_neg for y < 0 (a CGMY-type measure; Sec. 2 and Sec. 4 allow
 * asymmetric measures); in 2D the symmetric kernel tilted along the first
 * axis, nu(y) = C exp(-lam0 |y| + theta y_1) / |y|^{2+2s} with
 * lam0 = (lambda + lambda_neg)/2, theta = (lambda_neg - lambda)/2 (the same
 * two rates along that axis).  The generator keeps the compensator of
 * equ:I1approx, int (u(x+y) - u(x) - rho(y) y.grad u(x)) nu(y) dy, whose u'
 * sum S1 = sum' w_k rho_k nu(kh) k_1 h no longer vanishes: it enters the
 * nearest neighbours along the first axis as a drift -S1 (central
 * difference); in 2D each axis has its own u'' coefficient (C2 - S2)/2. */
/* VARIABLE_ORDER: the row of the point x_i takes its own jump index
 * s_i = s_field[i]: nu_i(y) = C_i exp(-lambda |y|) / |y|^{d+2 s_i} with
 * C_i = C when C > 0, else c_{d,s_i} (lambda = 0: the variable-order
 * fractional Laplacian -(-Delta)^{s(x)} of Sec. 5.4, eq. equ:2dmodel).  Each
 * row is the TEMPERED row of Sec. 4 at its own s_i (quadrature constants
 * S0, S2, C2, T computed once per distinct value of s_field), so the
 * generator is neither Toeplitz nor symmetric.  The field p.s is ignored. */

/* The model problem (Sec. 3.1 eq. equ:ut; Sec. 4 eqs. equ:ny2 and the
 * zero-exterior remark).  Domain: the box [lo, hi]^dim, u = 0 outside; in 2D
 * a mask can take grid points out of the domain (u = 0 there too: the
 * generator of a masked domain is the box generator's rows and columns of
 * the points kept), e.g. the L-shaped domain [-1, 1]^2 without [0, 1]^2 of
 * Sec. 5.4.  With a mask the unknowns are the kept points in increasing
 * grid index p*n + q, N = number of kept points, and every vector of the
 * other calls is in that order.  mask and s_field are host arrays the
 * library reads during the call that takes the problem (it keeps copies);
 * the hlevy_server and hlevy_exterior_forcing* calls take neither. */
typedef struct {
  int32_t dim;       /* 1 or 2 */
  int32_t n;         /* interior grid points per axis, h = (hi - lo)/(n + 1); N = n^dim (mask: kept points) */
  double lo, hi;     /* box */
  double a;          /* diffusion coefficient (a >= 0): sigma^2/2 of the Levy triplet */
  double b[2];       /* drift (b[1] ignored in 1D) */
  double c;          /* killing rate (c <= 0) */
  double s;          /* jump index, 0 < s < 1 */
  double lambda;     /* tempering rate >= 0; 0 = fractional Laplacian kernel */
  double C;          /* kernel constant; C <= 0 selects c_{d,s} = 4^s G(d/2+s)/(pi^{d/2}|G(-s)|) */
  double r0;         /* singular window radius rho (snapped to round(r0/h) h); Sec. 5.3 uses 0.2 */
  int32_t kernel;    /* hlevy_kernel; GAUSSIAN ignores s, lambda and r0, and C <= 0 selects 1 */
  int32_t pad;
  double eps2;       /* GAUSSIAN: eps^2 > 0 of nu(y) = C exp(-eps2 |y|^2) */
  double lambda_neg; /* TEMPERED_ASYM: tempering rate >= 0 of the jumps y < 0 (lambda: y > 0) */
  const uint8_t* mask;   /* NULL, or (2D) n*n bytes in grid order, nonzero = point in the domain */
  const double* s_field; /* VARIABLE_ORDER: N jump indices in (0, 1), natural order; else NULL */
} hlevy_problem;

/* H-matrix parameters (App. B.1): leaf size N_min, admissibility eta
 * (eq. equ:adm), N_block = ceil(N/N_max), ACA tolerance and rank capacity
 * of a low-rank block; the tile shapes of the per-step products (0 picks
 * them from the operator; hlevy_autotune times the alternatives), and what
 * a factorisation does when a rounded addition needs more than the rank
 * capacity. */
typedef struct {
  int32_t leaf;      /* max points per leaf cluster (N_min), 16..64 */
  double eta;        /* admissibility constant, > 0 */
  int32_t n_block;   /* N_max = ceil(N / n_block); >= 1.  With ACA (taylor_rank 0) an admissible
                        block has at most 16384 rows, so n_block >= N / 16384 */
  double aca_tol;    /* relative Frobenius tolerance of the far-field blocks */
  int32_t max_rank;  /* rank capacity of a low-rank block, 4..32 */
  int32_t gather_waves;    /* wavefronts per gather workgroup: 0 (8 single, 4 batched), 4 or 8 */
  int32_t rank_bucket;     /* register width of the low-rank product kernels: 0 (from the ranks), 8, 16 or 32 */
  int32_t strict_rank_cap; /* 1: an FP64 factorisation whose rounded additions overflow the rank
                              capacity fails with HLEVY_ERR_RANK_CAP; 0: the blocks are truncated
                              at the capacity, counted in hlevy_fac_info.rank_overflows, and the
                              refinement's residual checks guard the solutions */
  int32_t taylor_rank;     /* GAUSSIAN kernel only: > 0 builds every admissible block from the first
                              taylor_rank terms of the Taylor expansion of Sec. 3.3 about its row
                              cluster's centre (2D: products of the 1D series in order of total
                              degree), stored at that fixed rank without truncation (the paper's
                              fixed-rank construction); <= max_rank.  Admissible blocks with fewer
                              than taylor_rank rows or columns are stored dense.  Required (> 0) for the
                              Gaussian kernel: partially pivoted ACA, whose stopping rule looks at
                              the last cross only, stops early on its 2D blocks (4.9 % block error
                              measured at eps2 = 5); 0 for the tempered kernel (ACA) */
  int32_t cluster;         /* hlevy_cluster: how a cluster is split in two (both keep the order of
                              the points inside each half) */
} hlevy_hparams;

/* Splitting rule of the cluster tree (App. B.1; Sec. 5.4 reorders by
 * recursive K-means with two clusters).  BISECT: 1D halves the index
 * range, 2D halves the longest side of the bounding box (ties: first
 * axis).  KMEANS: Lloyd's iteration for two centres on the integer grid
 * coordinates of the cluster's points, started from the first point of
 * smallest and the first of largest coordinate along the longest side;
 * a point joins the second centre only when strictly nearer to it; at most
 * 64 iterations, stopping when no point moves; distances compared exactly
 * (integer arithmetic), so the tree does not depend on rounding.  KMEANS
 * needs N <= 2^22. */
typedef enum { HLEVY_CLUSTER_BISECT = 0, HLEVY_CLUSTER_KMEANS = 1 } hlevy_cluster;

/* Iterative refinement of a solve M x = b preconditioned by the H-LU
 * (Sec. 5.1 uses the H-LU inverse as a preconditioner): after the direct
 * solve x = U^{-1} L^{-1} b, `sweeps` sweeps x <- x + U^{-1} L^{-1} (b - M x)
 * with the FP64 operator in the residual.  At a check the relative residual
 * ||b - M x||_2 / ||b||_2 of the current x is measured on the device (one
 * more product with G, read back on the host); while it is above `tol`
 * further sweeps run, up to `max_sweeps` sweeps in all, and a check that
 * still misses `tol` fails the call with HLEVY_ERR_NOT_CONVERGED. */
typedef struct {
  double tol;          /* relative residual target; <= 0: no target (checks only measure) */
  int32_t sweeps;      /* sweeps per solve / per Crank-Nicolson step (fixed count) */
  int32_t check_every; /* hlevy_step: check every k-th step and the last; 0: the last step only */
  int32_t max_sweeps;  /* most sweeps at a check that misses tol (values below `sweeps` mean `sweeps`) */
  int32_t pad;
} hlevy_refine;

/* Outcome of a solve or stepping call.  Filling it synchronises the stream. */
typedef struct {
  int64_t steps_done;          /* completed steps (solves: right-hand sides) */
  double last_rel_residual;    /* at the last check, -1 when none was made */
  double max_rel_residual;     /* largest measured in the call, -1 when none */
  int32_t checks;              /* residual checks made */
  int32_t max_sweeps_used;     /* most sweeps a checked solve or step took */
  int32_t rank_overflows;      /* low-rank blocks of the factor truncated at their capacity */
  int32_t pad;
  double seconds;              /* host wall time of the call */
} hlevy_stats;

/* Structure summary, computed on the host (no device needed). */
typedef struct {
  int64_t N;
  int32_t depth;              /* levels of the cluster tree below the root */
  int32_t n_clusters;
  int32_t n_dense;            /* inadmissible leaves (dense) */
  int32_t n_lowrank;          /* admissible leaves (low rank) */
  int32_t max_leaf_points;
  int32_t min_leaf_points;
  int64_t dense_entries;      /* sum of m*n over dense leaves */
} hlevy_plan_info_t;

typedef struct {
  int64_t dense_entries;      /* stored FP64 entries in dense leaves */
  int64_t lowrank_entries;    /* stored entries sum (m+n)*k over low-rank leaves */
  int32_t max_rank;
  double mean_rank;
  int32_t rank_overflows;     /* low-rank blocks truncated at their capacity (0: see subdivided_blocks) */
  int32_t subdivided_blocks;  /* admissible blocks subdivided or kept dense for the rank cap */
  size_t device_bytes;        /* device memory the operator holds */
} hlevy_op_info_t;

typedef struct {
  size_t device_bytes;        /* device memory the factor holds (the operator's not included) */
  int32_t rank_overflows;     /* rounded additions of the H-LU truncated at the rank capacity */
  int32_t max_rank;           /* largest rank of a low-rank block of L^{-1} or U^{-1} */
  double product_bytes[3];    /* stored bytes read by one product with G, L^{-1}, U^{-1} */
  double lu_tol, dt;
  int32_t prec, pad;
} hlevy_fac_info_t;

typedef struct hlevy_op hlevy_op;
typedef struct hlevy_fac hlevy_fac;

/* Device memory supplied by the caller: alloc(bytes, ctx) returns device
 * memory aligned to 256 bytes, or NULL on failure (the call then fails with
 * HLEVY_ERR_OOM); free(p, ctx) releases it.  An operator assembled with an
 * allocator takes all its storage and the transient buffers of its calls
 * from it, and so does every factor of that operator; buffers are freed
 * through the same allocator when the handle is destroyed.  The allocator
 * must stay valid until then.  NULL: hipMalloc / hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* p, void* ctx);
  void* ctx;
} hlevy_allocator;

/* Library ABI version (HLEVY_ABI_VERSION). */
int32_t hlevy_abi_version(void);

/* Thread-local message of the last failed call on this thread. */
const char* hlevy_last_error(void);

/* Host only: build the cluster tree (1D index halving, 2D geometric
 * bisection of the longest box side, App. B.1) and the block tree with the
 * admissibility of eq. equ:adm on point bounding boxes, and report counts.
 * Errors: HLEVY_ERR_INVALID_ARG for an invalid descriptor. */
hlevy_status hlevy_plan_info(const hlevy_problem* prob, const hlevy_hparams* hp,
                             hlevy_plan_info_t* out);

/* Resident device bytes of an operator assembled from (prob, hp) plus one
 * factor of precision prec: the memory hlevy_assemble and hlevy_factor keep
 * until the handles are destroyed (hlevy_op_info / hlevy_fac_info report
 * the actual bytes).  The transient workspace of a factorisation (at most
 * workspace_bytes of hlevy_factor_batched) is not included.  Computed on the
 * host from the block structure (App. B.1) with every low-rank block at its
 * rank capacity, so it bounds the actual bytes from above, unless the
 * assembly subdivides blocks whose compression needs more than the rank
 * capacity (hlevy_op_info.subdivided_blocks > 0): those are known only after
 * the ACA and their dense storage is not included.  Errors:
 * HLEVY_ERR_INVALID_ARG for an invalid descriptor or precision. */
hlevy_status hlevy_footprint(const hlevy_problem* prob, const hlevy_hparams* hp, int32_t prec,
                             size_t* bytes_out);

/* Assemble the generator G as an H-matrix on the device: quadrature constants
 * (Sec. 4, equ:I1approx - equ:I3approx), dense near-field leaves (Sec. 4 row
 * form, eq. equ:Aij local terms), partially pivoted ACA of every admissible
 * block followed by truncation to aca_tol (App. B.1).  A block whose
 * truncation needs more than max_rank columns is subdivided into its four
 * sub-blocks (admissible in turn), or stored dense when its clusters are
 * leaves, and the problem is assembled again with that structure, so no
 * block is truncated at its capacity.  *out receives a new handle.  alloc:
 * the caller's allocator or NULL.  Synchronises `stream`. */
hlevy_status hlevy_assemble(const hlevy_problem* prob, const hlevy_hparams* hp,
                            const hlevy_allocator* alloc, void* stream, hlevy_op** out);

/* Batched worklist: assemble `count` problems (probs[i] with hps[i]) as
 * hlevy_assemble does, with the quadrature, near-field and ACA kernels of
 * all problems enqueued back to back and the truncation of every ACA block
 * in one plan (problems of equal aca_tol share its launches); each out[i]
 * is the same operator hlevy_assemble gives.  On error every out[i] is NULL
 * and nothing is leaked.  Synchronises `stream`. */
hlevy_status hlevy_assemble_batched(const hlevy_problem* probs, const hlevy_hparams* hps, int32_t count,
                                    const hlevy_allocator* alloc, void* stream, hlevy_op** out);

/* Copy the quadrature constants S0, S2, C2, T (Sec. 4) and S1 (the u' sum of
 * an asymmetric measure, 0 otherwise) to host `out`; for a 2D asymmetric
 * measure S2 and C2 are those of the first axis.  Synchronises `stream`. */
hlevy_status hlevy_op_constants(const hlevy_op* op, double out[5], void* stream);

/* Forcing of a non-zero exterior, tempered kernels (Sec. 4: the terms of
 * equ:I1approx - equ:I3approx that reach outside the box; the far-field term
 * f^{L_W} of equ:I2approx collects what lies beyond the window).  For
 * u = u_ext outside the box, the scheme on the box is G u + g: g (device,
 * natural order, length n) takes, in row i, the window offsets k
 * (|k| <= NW = n + 1) whose point x_i + kh is exterior, each with W_k nu(kh)
 * (W_k = h, h/2 at |k| = NW), and the local terms on the exterior neighbours
 * lo and hi.  u_ext (device, 2 NW values): lattice points lo - (NW-1)h .. lo
 * ascending, then hi .. hi + (NW-1)h.  2D: u_ext holds the extended lattice
 * of indices -NW .. n - 1 + NW per axis, (3n + 2)^2 values in grid order
 * (first coordinate slowest; the n^2 interior entries are ignored), and row
 * (p, q) takes every exterior point of its window (|k|_inf <= NW) with
 * W_k1 W_k2 nu(kh) and the local terms of its exterior nearest neighbours.
 * The integral of u_ext beyond the window (|y| > L_W) is not included (its
 * -u T part is in G; hlevy_exterior_forcing_far adds it).  A time-independent
 * exterior enters hlevy_step as g with phi = 1.  Errors:
 * HLEVY_ERR_INVALID_ARG for a Gaussian, variable-order or masked operator
 * or overlapping buffers.  Synchronises `stream`. */
hlevy_status hlevy_exterior_forcing(const hlevy_op* op, const double* u_ext, double* g, void* stream);

/* Forcing of a non-zero exterior with its far field, tempered kernels:
 * g + f, with g as hlevy_exterior_forcing (from the lattice points of the
 * window nearest the box) and f the far-field term f^{L_W} of equ:I2approx
 * (eq. equ:fxy), which the paper leaves to an input or a quadrature.
 * 1D: row i takes the trapezoid rule over the lattice offsets
 * k = NW .. next (NW = n + 1), each side with its own kernel (nu(kh) to the
 * right, nu(-kh) to the left) and weights h, h/2 at k = NW and k = next
 * (nothing when next = NW); beyond next h the exterior is the constant
 * tail_right (y > 0) or tail_left (y < 0), times the integral of nu over
 * that half line (incomplete gamma function, each side with its rate).
 * u_ext (device, 2 next values): lattice points lo - (next-1)h .. lo
 * ascending, then hi .. hi + (next-1)h; n + 1 <= next <= 2^26.
 * 2D: row (p, q) takes the product trapezoid rule over the square
 * |k|_inf <= next (weights h, h/2 at |k_a| = next) less the window's
 * (|k|_inf <= NW, h/2 at |k_a| = NW), so only lattice points with
 * |k|_inf >= NW enter; beyond the square the exterior is the constant
 * tail_right (y1 > 0) or tail_left (y1 < 0), times the measure of that
 * half of the region |y|_inf > next h (polar coordinates: Gauss-Legendre
 * in the angle, the incomplete gamma function in the radius; the tilted
 * measure with its angle-dependent rate).  u_ext (device,
 * (n + 2 next)^2 values): the extended lattice of indices
 * -next .. n - 1 + next per axis, first coordinate slowest; entries inside
 * the box are not read; n + 1 <= next <= 2^13.  Work: O(n * next) in 1D,
 * O(n^2 * next^2) in 2D (every row sums its whole extended square), and a
 * device table of (2 next + 1)^2 doubles in 2D.
 * With next = n + 1 and zero tails the result is hlevy_exterior_forcing's;
 * with a constant exterior c (tails c) G c + g + f = 0 in every row.
 * Errors as hlevy_exterior_forcing, and HLEVY_ERR_INVALID_ARG for next out
 * of range or non-finite tails.  Synchronises `stream`. */
hlevy_status hlevy_exterior_forcing_far(const hlevy_op* op, const double* u_ext, int32_t next, double tail_left,
                                        double tail_right, double* g, void* stream);

/* Storage summary of the assembled operator.  Synchronises `stream`. */
hlevy_status hlevy_op_info(const hlevy_op* op, hlevy_op_info_t* out, void* stream);

/* Storage summary of a factor.  Synchronises `stream`. */
hlevy_status hlevy_fac_info(const hlevy_fac* fac, hlevy_fac_info_t* out, void* stream);

/* y = G x (App. B.2: dense leaves by GEMV, low-rank leaves as U (V^T x)).
 * x, y: device, length N, natural order, must not alias. */
hlevy_status hlevy_matvec(const hlevy_op* op, const double* x, double* y, void* stream);

/* Write the H-matrix G densely: dense[i*N + j] = G_ij in natural order
 * (row-major).  `dense` is a device buffer of N*N doubles; meant for tests
 * at small N. */
hlevy_status hlevy_op_densify(const hlevy_op* op, double* dense, void* stream);

/* Factor M = I - dt/2 G by H-LU (App. B.3) and form the H-inverses of its
 * triangular factors, truncating every low-rank addition at lu_tol.
 * prec = HLEVY_PREC_FP64 keeps FP64 factors; HLEVY_PREC_MIXED stores the
 * inverse factors in FP32 for the refinement preconditioner,
 * HLEVY_PREC_MIXED_BF16 their low-rank leaves in BF16 (the factorisation
 * itself runs in FP64 arithmetic on every path).  The factor
 * keeps a reference to `op` (op must outlive it).  Independent parts of the
 * factorisation run on two further streams that the library keeps per host
 * thread and device (default priority, created on first use, never
 * destroyed); their work joins `stream` before the call returns.
 * Synchronises `stream`. */
hlevy_status hlevy_factor(const hlevy_op* op, double dt, int32_t prec, double lu_tol,
                          void* stream, hlevy_fac** out);

/* Batched worklist: factor M_i = I - dt[i]/2 G_i of `count` independent
 * problems (ops[i], each assembled by hlevy_assemble) in one plan.  The H-LU
 * recursion of App. B.3 runs jointly over the problems, aligned from the
 * leaves upwards, so every batch of products, copies and rounded additions
 * is one launch for all of them (a problem's result is the same as with
 * hlevy_factor).  Problems are taken in groups whose factorisation memory
 * fits `workspace_bytes` (0 = 48 GiB); each group is one plan.  prec and
 * lu_tol as for hlevy_factor, common to all problems.  out[i] receives
 * problem i's factor (each used and destroyed on its own).  A group shares
 * its zero-pivot flag and rank-overflow count.  Uses the library's two
 * further streams as hlevy_factor does.  On error every out[i] is NULL and
 * nothing is leaked.  Synchronises `stream`. */
hlevy_status hlevy_factor_batched(const hlevy_op* const* ops, const double* dt, int32_t count,
                                  int32_t prec, double lu_tol, size_t workspace_bytes,
                                  void* stream, hlevy_fac** out);

/* Solve M X = B for nrhs right-hand sides (App. B.3 forward and backward
 * solve): x = U^{-1} (L^{-1} b) through the H-inverses of the factors, then
 * iterative refinement as hlevy_refine describes.  b, x: device, natural
 * order, column c at b + c*ld (ld >= N), must not overlap.  Right-hand
 * sides are taken up to four at a time: each product then reads the factor
 * once for all of them.  refine may be NULL: 2 sweeps (mixed) or 1 sweep
 * (FP64; products with explicit inverse factors lose accuracy like
 * eps cond(L) cond(U), about 1e-6 relative residual at N = 65536, and one
 * sweep restores about 1e-12), no target.  A check is made on every column
 * when refine->tol > 0 or stats is given; stats reports the largest
 * residual over the columns.  On HLEVY_ERR_NOT_CONVERGED x is unchanged. */
hlevy_status hlevy_solve(hlevy_fac* fac, const double* b, double* x, int64_t nrhs, int64_t ld,
                         const hlevy_refine* refine, hlevy_stats* stats, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): hlevy_solve for
 * one right-hand side (nrhs = 1) that allocates nothing.  Its work vectors
 * and check slots live in a static device array of the library,
 * 4 * HLEVY_NOALLOC_MAX_N + 514 doubles (about 8 MiB) on every device it
 * runs on, held until the process ends; N above HLEVY_NOALLOC_MAX_N fails
 * with HLEVY_ERR_INVALID_ARG.  Every call on a device shares that array:
 * calls that overlap on one device (other streams, other host threads)
 * race and must be serialised by the caller.  b, x, refine, stats and the
 * result are as for hlevy_solve with nrhs = 1 (the same kernels, the same
 * arithmetic); synchronises `stream` only when a residual check is made. */
#define HLEVY_NOALLOC_MAX_N 262144
hlevy_status hlevy_solve_noalloc(hlevy_fac* fac, const double* b, double* x, const hlevy_refine* refine,
                                 hlevy_stats* stats, void* stream);

/* Autotuner of the leaf size and the tile shapes of the per-step products
 * (the batched worklist's "autotuned leaf and tile sizes"): for the problem
 * and the caller's parameters `base`, every candidate of leaf {64, 32} x
 * gather_waves {0, 4, 8} x rank_bucket {0, 16} (base's own values first)
 * is assembled, factored (prec, lu_tol) and stepped on the device; the
 * objective is the whole job per problem, assembly + factorisation +
 * nsteps steps at the measured rate (one refinement sweep per step).  With
 * batch > 1 the candidates run through the batched entry points on
 * min(batch, 8) copies, so the batched kernels are the ones timed.  The
 * fastest candidate is returned in out (leaf, gather_waves, rank_bucket;
 * the other fields of base are kept by the caller) with its objective and
 * that of base.  cache_path (NULL: none) names a JSON file of earlier
 * choices keyed by dimension, N rounded to a power of two, precision and
 * batched-or-single: a key found there is returned without device work
 * (from_cache = 1), a new choice is added to it.  Synchronises `stream`.
 * Errors: HLEVY_ERR_INVALID_ARG for invalid arguments or an unwritable
 * cache; errors of the trial calls as they return them. */
#define HLEVY_TUNE_MAX_CAND 16
typedef struct {
  int32_t leaf, gather_waves, rank_bucket; /* the fastest candidate */
  int32_t from_cache;                      /* 1: read from the cache, nothing timed */
  int32_t ncand, pad;                      /* candidates timed */
  double seconds;                          /* its whole job per problem */
  double default_seconds;                  /* base's whole job per problem */
  int32_t cand_leaf[HLEVY_TUNE_MAX_CAND], cand_gather_waves[HLEVY_TUNE_MAX_CAND],
      cand_rank_bucket[HLEVY_TUNE_MAX_CAND];
  double cand_seconds[HLEVY_TUNE_MAX_CAND];
} hlevy_tune_result;

hlevy_status hlevy_autotune(const hlevy_problem* prob, const hlevy_hparams* base, double dt, int32_t prec,
                            double lu_tol, int64_t nsteps, int32_t batch, const char* cache_path, void* stream,
                            hlevy_tune_result* out);

/* Advance u (device, natural order, in/out) by nsteps Crank-Nicolson steps
 * of eq. equ:scheme with forcing f(x, t_n) = phi[n] g(x):
 *   M u^{n+1} = (I + dt/2 G) u^n + dt/2 (phi[n] + phi[n+1]) g.
 * g: device vector or NULL (no forcing); phi: host array of nsteps+1 values
 * (ignored when g is NULL).  Each step solves M w = 2 u^n + F_n with
 * refinement (hlevy_refine) and sets u^{n+1} = w - u^n.  Residual checks
 * (refine->tol > 0, or stats given) run on every check_every-th step and on
 * the last one.  A step whose check misses refine->tol after max_sweeps
 * sweeps is not applied: the call returns HLEVY_ERR_NOT_CONVERGED with u at
 * the last completed step and stats->steps_done counting the completed
 * steps.  stats may be NULL. */
hlevy_status hlevy_step(hlevy_fac* fac, double* u, int64_t nsteps, const double* g,
                        const double* phi, const hlevy_refine* refine,
                        hlevy_stats* stats, void* stream);

/* Batched worklist: advance u[i] (device, natural order, in/out) of the
 * `count` problems facs[i] by nsteps[i] Crank-Nicolson steps each, without
 * forcing (eq. equ:scheme with f = 0), each with its own dt.  Every product
 * of a step is one projection and one gather launch over all problems (per
 * group of equal rank bucket), so small problems share the chip.  Sweeps
 * per step: refine->sweeps, or when refine is NULL the largest default of
 * hlevy_step among the factors.  The factors must be distinct (each one's
 * work vectors are used); the result of each problem is the same as
 * hlevy_step on it alone.  With refine->tol > 0 or stats given, the last
 * step of every problem measures its relative residual (no further sweeps);
 * stats reports the largest, and the call returns HLEVY_ERR_NOT_CONVERGED
 * when one is above refine->tol (every u[i] is advanced all the same).
 * Synchronises `stream`. */
hlevy_status hlevy_step_batched(hlevy_fac* const* facs, double* const* u, const int64_t* nsteps, int32_t count,
                                const hlevy_refine* refine, hlevy_stats* stats, void* stream);

/* Steady solves (shift I - G) x = b by a Krylov iteration that the factor
 * preconditions: Sec. 5.1 uses the factorised H-matrix as the
 * preconditioner of an iteration with the H-matrix, Sec. 5.3 solves the
 * fractional Poisson problem (shift = 0, fractional generator) by conjugate
 * gradients, Sec. 5.4 tracks the relative residual of eq.
 * equ:relative_error over the iterations.  The operator products use G in
 * FP64 (the factor's operator); the preconditioner is z = U^{-1} L^{-1} r
 * with the factor's inverse factors, a good one when the factor's
 * M = I - dt/2 G is close to a multiple of shift I - G, i.e. 2/dt near
 * shift (for shift = 0: dt large against 1/lambda_min(-G)).  Methods:
 * HLEVY_KRYLOV_CG for a symmetric positive definite shift I - G (symmetric
 * jump kernel, no drift), HLEVY_KRYLOV_BICGSTAB and HLEVY_KRYLOV_GMRES
 * (restarted, right-preconditioned: the residual it minimises is that of
 * the unpreconditioned system; Gram-Schmidt applied twice; the Givens
 * rotations and the small least-squares problem on the host) for any
 * operator.  Deterministic: every reduction runs in a fixed order. */
typedef enum { HLEVY_KRYLOV_CG = 0, HLEVY_KRYLOV_BICGSTAB = 1, HLEVY_KRYLOV_GMRES = 2 } hlevy_krylov_method;
typedef struct {
  int32_t method;        /* hlevy_krylov_method */
  int32_t max_iter;      /* >= 1 */
  double tol;            /* stop when ||b - A x||_2 <= tol ||b||_2 (recursive residual), A = shift I - G */
  double shift;
  int32_t precondition;  /* 1: with the factor's inverse factors; 0: none (for comparison) */
  int32_t use_guess;     /* 1: x holds the initial guess on entry; 0: start from x = 0 */
  const hlevy_op* op;    /* the operator G of A: NULL = the factor's own; else an operator of the same
                            cluster tree ordering (same problem and tree parameters, e.g. a tighter
                            aca_tol), so that a coarse factor preconditions an accurate operator as
                            in Sec. 5.4 (preconditioner from eps1 = 1e-4, iteration on A) */
  int32_t restart;       /* GMRES: Arnoldi steps per cycle, 1..64 (0: 30); ignored otherwise */
  int32_t pad;
} hlevy_krylov;
typedef struct {
  int32_t iterations;    /* iterations taken (a BiCGSTAB iteration is two products with G) */
  int32_t converged;     /* 1 when tol was met */
  double rel_residual;   /* ||b - A x||_2 / ||b||_2 recomputed from the returned x */
  double seconds;        /* wall time of the call */
} hlevy_krylov_stats;

/* b, x: device, length N, natural order, must not overlap.  history: NULL
 * or a host array of max_iter + 1 doubles that receives the recursive
 * relative residual before the first iteration and after each one (entries
 * past the last iteration are not written).  x receives the last iterate
 * also when tol is not met; the call then returns HLEVY_ERR_NOT_CONVERGED
 * (stats filled).  A zero right-hand side gives x = 0 after no iteration.
 * Errors: HLEVY_ERR_INVALID_ARG for a bad option or overlapping b and x.
 * Synchronises `stream` once per iteration (twice for BiCGSTAB; GMRES once
 * per Arnoldi step and once per restart). */
hlevy_status hlevy_krylov_solve(hlevy_fac* fac, const double* b, double* x, const hlevy_krylov* opt,
                                hlevy_krylov_stats* stats, double* history, void* stream);

/* Serving loop.  Requests (a problem, dt, a horizon of nsteps unforced
 * Crank-Nicolson steps, u0) arrive at any time; each hlevy_server_poll is
 * one scheduling round:
 *  1. admission in arrival order while the resident memory (cached
 *     operators and factors, request state) fits hbm_budget; idle cached
 *     operators are evicted least recently used first; a request waits
 *     when memory is short (one request is always admitted when nothing
 *     else is active);
 *  2. operators not in the cache are assembled and factored in one joint
 *     plan (hlevy_factor_batched); requests with equal problem, hparams and
 *     dt share one cached factor.  When the device runs out of memory here,
 *     every idle cached operator is evicted and the factorisation runs once
 *     more; if that fails too while other requests are active, the round's
 *     new requests return to the head of the queue and no new operator is
 *     admitted until a cached one falls idle;
 *  3. every active request (at most max_active) advances by
 *     min(chunk, its steps left) steps in one batched loop
 *     (hlevy_step_batched's products; each request keeps its own vectors;
 *     a request whose steps are done sits out the rest of the loop);
 *  4. finished requests get u^{nsteps} written to their u_out; the last
 *     step of every request measures its relative residual (stats).
 * Submission validates the problem as hlevy_assemble does.
 * A request's result equals hlevy_step with a factor of the same
 * parameters (same arithmetic, summation order of the batched products).
 * The server's calls are not thread safe. */
typedef struct {
  size_t hbm_budget;   /* resident bytes allowed; 0 = 64 GiB.  A round that factors new operators
                          also takes a transient workspace from the memory then free (at most
                          48 GiB), so the budget should leave room for it */
  int32_t prec;        /* HLEVY_PREC_MIXED or HLEVY_PREC_FP64 */
  double lu_tol;       /* H-LU truncation of the factors */
  int32_t sweeps;      /* refinement sweeps per step */
  int32_t chunk;       /* CN steps per scheduling round, >= 1 */
  int32_t max_active;  /* most requests advanced together, >= 1 */
  double tol;          /* relative residual target of a request's last step; <= 0: measured only */
} hlevy_server_config;

typedef struct {
  int64_t submitted, completed, active, queued;
  int64_t cache_hits, cache_misses, evictions, cached_operators;
  int64_t problem_steps;        /* CN steps advanced, summed over requests */
  size_t bytes_in_use;          /* resident bytes: cached operators with their factors (the hlevy_footprint
                                   estimate until built, then the bytes allocated) and request state */
  double assemble_seconds, factor_seconds, step_seconds;
  int64_t failed;               /* requests whose operator could not be built */
  int64_t not_converged;        /* completed requests whose last-step residual missed tol */
  double max_rel_residual;      /* largest last-step residual of a completed request, -1 before any */
} hlevy_server_stats;

typedef struct hlevy_server hlevy_server;

/* New server; its device work goes to `stream`.
 * Errors: HLEVY_ERR_INVALID_ARG for a bad configuration. */
hlevy_status hlevy_server_create(const hlevy_server_config* cfg, void* stream, hlevy_server** out);

/* Queue a request.  u0: device, natural order, copied on `stream` before the
 * call returns (the caller may reuse it); u_out: device, natural order,
 * length N, must stay valid until the request is reported done.  *id
 * receives the request's id.  Errors: HLEVY_ERR_INVALID_ARG for an invalid
 * problem or dt. */
hlevy_status hlevy_server_submit(hlevy_server* srv, const hlevy_problem* prob, const hlevy_hparams* hp,
                                 double dt, int64_t nsteps, const double* u0, double* u_out, int64_t* id);

/* One scheduling round (see above); synchronises the stream.  Writes up to
 * `cap` ids of finished requests to done_ids and their count to *ndone
 * (more are returned by later calls). */
hlevy_status hlevy_server_poll(hlevy_server* srv, int64_t* done_ids, int32_t cap, int32_t* ndone);

/* Requests that failed: when the assembly or factorisation of the operators
 * new in a round fails (other than for device memory while other requests
 * are active, see above), hlevy_server_poll returns that error and those
 * requests leave the server (their u_out is not written).  Writes up to
 * `cap` of their ids to ids and the count to *n. */
hlevy_status hlevy_server_take_failed(hlevy_server* srv, int64_t* ids, int32_t cap, int32_t* n);

/* Counters of the server. */
hlevy_status hlevy_server_stats_get(hlevy_server* srv, hlevy_server_stats* out);

/* Frees every cached operator and factor and every queued request. */
void hlevy_server_destroy(hlevy_server* srv);

/* y = A x with one of the matrices the factor applies every step, in the
 * storage precision of the factor: which = 0: the generator G of the
 * residual operator (FP64 on both paths), 1: L^{-1}, 2: U^{-1} (App. B.2
 * product on the H-inverses of the factors of M = I - dt/2 G; FP32 on the
 * mixed path).
 * x, y: device, length N, natural order, must not alias.
 * Errors: HLEVY_ERR_INVALID_ARG for null pointers, aliasing or a bad `which`. */
hlevy_status hlevy_fac_apply(hlevy_fac* fac, int32_t which, const double* x, double* y, void* stream);

/* Kernel timing of the per-step matrix-vector products (roofline
 * reporting).  Runs `reps` rounds of the three products of a Crank-Nicolson
 * step in stepping order -- G, L^{-1}, U^{-1} -- on internal vectors, each
 * product's two kernels (projection t = V^T x of the low-rank leaves, then
 * the gather y = D x + U t per leaf cluster) bracketed by HIP events on
 * `stream`.  Index w of each array: 0 = G, 1 = L^{-1}, 2 = U^{-1}.
 * Synchronises `stream`; errors: HLEVY_ERR_INVALID_ARG for reps outside
 * [1, 100000]. */
typedef struct {
  int64_t N;
  int32_t reps, pad;
  double project_ms[3];     /* mean projection kernel time */
  double gather_ms[3];      /* mean gather kernel time */
  double dense_bytes[3];    /* stored dense-leaf bytes (read by the gather) */
  double u_bytes[3];        /* low-rank U factor bytes (read by the gather) */
  double v_bytes[3];        /* low-rank V factor bytes (read by the projection) */
  double partial_bytes[3];  /* projection partials (written, then read by the gather) */
} hlevy_kernel_times;

hlevy_status hlevy_fac_kernel_times(hlevy_fac* fac, int32_t reps, void* stream, hlevy_kernel_times* out);

void hlevy_op_destroy(hlevy_op* op);
void hlevy_fac_destroy(hlevy_fac* fac);

#ifdef __cplusplus
}
#endif
#endif /* HLEVY_H */
