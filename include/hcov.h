/*
 * hcov -- H-matrix Gaussian log-likelihood of a Matérn random field on an
 * AMD Instinct MI355X (gfx950).  C ABI: plain pointers and sizes only.
 *
 * The method is the one of Litvinenko, Kriemann, Genton, Sun and Keyes,
 * "HLIBCov: Parallel hierarchical matrix approximation of large covariance
 * matrices and likelihoods with applications in parameter identification",
 * arXiv:1709.08625 (cited below as [HLIBCov]):
 *   - joint Gaussian log-likelihood, Eq. (1) of Sec. 1;
 *   - its H-matrix form through the H-Cholesky factor, Eq. (2) of Sec. 1;
 *   - Matérn covariance, Eq. (3) of Sec. 2.1, theta = (ell, nu, sigma^2);
 *   - cluster tree / block cluster tree / admissibility, Sec. 2.2 and
 *     Appendix A (standard admissibility Adm_eta);
 *   - fixed-accuracy low-rank blocks ||M - M~|| <= eps ||M||, Sec. 2.2;
 *   - ACA with SVD recompression, the remark at the end of Appendix B;
 *   - nugget tau^2 added to the diagonal, Sec. 4 and Sec. 5.2.
 *
 * Conventions for every call:
 *   - Return value: HCOV_OK (0) or a negative error code; hcov_strerror()
 *     names it and hcov_last_error() holds a message for the context.  No C++
 *     exception crosses this boundary.
 *   - Vectors z, x passed to the context are in the caller's (external) point
 *     order; the library applies its cluster permutation internally.
 *   - "where" arguments: HCOV_HOST (host memory) or HCOV_DEVICE (device
 *     memory on the context's GPU).
 *   - A context is not thread safe; distinct contexts are independent.  All
 *     device work of a context is ordered on its HIP stream.
 *   - Device memory of a context comes from the allocator callbacks in
 *     hcov_opts when given (e.g. the PyTorch caching allocator), else from
 *     hipMalloc; it is released by hcov_destroy.
 */
#ifndef HCOV_H_
#define HCOV_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ return codes */
#define HCOV_OK 0
#define HCOV_EINVAL -1      /* argument out of its domain (theta, eps, n, ...) */
#define HCOV_ENOTSPD -2     /* non-positive or non-finite pivot in H-Cholesky */
#define HCOV_ENOMEM -3      /* device or host allocation failed / over cap */
#define HCOV_ESTATE -4      /* call out of order (e.g. logdet before cholesky) */
#define HCOV_EDEVICE -5     /* HIP runtime error or no device */
#define HCOV_ERANK -6       /* a low-rank block needed more than max_rank */
#define HCOV_EAGAIN -7      /* serving: the request has not completed yet */

#define HCOV_HOST 0
#define HCOV_DEVICE 1

#define HCOV_FP64 0         /* every step in FP64 */
#define HCOV_MIXED 1        /* low-rank factors/updates FP32; diagonal, logdet, quad FP64;
                               low-rank truncations at max(eps, 1e-6) */

/* Matérn parameters, Eq. (3) [HLIBCov Sec. 2.1], with named fields:
 * sigma2 = sigma^2 > 0 (variance), ell > 0 (range; the kernel argument is
 * h/ell exactly as in Eq. (3)), nu > 0 (smoothness), nugget = tau^2 >= 0
 * added to the diagonal only [HLIBCov Sec. 5.2]. */
typedef struct {
  double sigma2;
  double ell;
  double nu;
  double nugget;
} hcov_theta;

typedef void* (*hcov_alloc_fn)(size_t bytes, void* user);
typedef void (*hcov_free_fn)(void* ptr, void* user);

/* Build options (all fields have defaults through hcov_opts_default). */
typedef struct {
  int precision;          /* HCOV_FP64 (default) or HCOV_MIXED */
  int max_rank;           /* capacity of every low-rank block (default 64) */
  double aca_eps_factor;  /* ACA stops at aca_eps_factor*eps before the SVD
                             recompression (default 0.1) */
  int fuse_solve;         /* 1: hcov_loglik solves L v = z inside the
                             factorisation sweep (default 1) */
  size_t mem_cap_bytes;   /* 0 = no cap; builds whose estimate exceeds it fail
                             with HCOV_ENOMEM */
  hcov_alloc_fn alloc;    /* optional device allocator; NULL = hipMalloc */
  hcov_free_fn free;
  void* alloc_user;
  int use_graphs;         /* 1: the factorisation sweep is captured once as a
                             HIP graph on a stream of the context and replayed
                             by later factorisations (default 1); 0: every
                             stage is launched separately */
  int oversample;         /* columns of a low-rank target's randomised sketch
                             in the factorisation's recompression beyond its
                             rank estimate (the larger of the block's assembled
                             rank and its rank hint, see hcov_cholesky);
                             default 10, range [2, 64]; the width is capped at
                             the block's room + 16 (max_rank + 16 unless
                             opts.initial_rank_cap sized the rooms) and at
                             min(rows, cols) of the block */
  int on_saturation;      /* HCOV_SAT_RETRY (default) or HCOV_SAT_ERROR: what a
                             saturated sketch does, see hcov_cholesky */
  int keep_matrix;        /* 1: keep a copy of the assembled C~ (dense and
                             low-rank arenas, about the size of the factor)
                             so that hcov_matvec, hcov_error_norms and the PCG
                             quadratic form work after the factorisation
                             (default 0; implied by HCOV_QUAD_PCG) */
  int quad_mode;          /* HCOV_QUAD_DIRECT (default): z^T C~^{-1} z as
                             v^T v with L~ v = z [Eq. (2)]; HCOV_QUAD_PCG:
                             z^T x with C~ x = z solved by conjugate
                             gradients on C~ preconditioned by L~ L~^T (the
                             listing of Appendix B) */
  double pcg_tol;         /* PCG stop: ||z - C~ x|| <= pcg_tol ||z|| (default
                             1e-6, the listing's tolerance) */
  int pcg_max_iter;       /* PCG iteration cap (default 150, the listing's) */
  int fixed_rank;         /* 0 (default): fixed accuracy eps; k > 0: every
                             low-rank block of C~ and of the factor keeps at
                             most k singular values above eps sigma_1 (the
                             fixed-rank H-matrices of Sec. 3, Tables 2 and 3);
                             k <= max_rank, and reaching it is no error */
  int adm_rule;           /* block admissibility [Appendix A]: HCOV_ADM_MIN
                             (default) the standard Adm_eta of Eq.
                             (stand_cond), min(diam) <= eta dist;
                             HCOV_ADM_MAX its max(diam) form; HCOV_ADM_WEAK
                             the weak admissibility Adm_W of Eq. (wead_adm):
                             every off-diagonal block of two different
                             clusters is low rank (eta unused) */
  int autotune;           /* 0 (default): every GEMM launch of the sweep runs
                             on the kernel the planner's cost model picks
                             (one 256-thread work-group per 64x64 tile, or
                             two lockstep groups per tile for launches bound
                             by their longest tile); 1: the context's first
                             factorisation is preceded by two factorisations
                             that time every launch where both kernels are
                             allowed, once with each, and each launch keeps
                             the faster kernel from then on (results differ
                             from the untuned ones by rounding only, and
                             repeat bit for bit after the tuning) */
  uint64_t seed;          /* seed of the Gaussian test matrix of the
                             randomised sketches (0, the default: the
                             library's fixed seed); other seeds give other
                             sketches and results that differ within the
                             truncation accuracy.  Every evaluation of a
                             context uses the same matrix. */
  int initial_rank_cap;   /* 0 (default): every low-rank block's U and V
                             arenas hold max_rank columns.  k in [1, max_rank]:
                             each block starts with room for k columns and is
                             grown (to at least twice its room and 5/4 of the
                             rank asked for, at most max_rank) when the ACA or
                             a truncation of the factorisation needs more; a
                             growth rebuilds the plan and the device buffers
                             and repeats the assembly and factorisation that
                             hit it, inside the same call (the results equal
                             those at full room up to rounding).  Capacities
                             only grow, over the life of the context.
                             HCOV_ERANK still means a block needs more than
                             max_rank.  A rebuild that does not fit
                             mem_cap_bytes or the device returns HCOV_ENOMEM
                             and leaves the context unusable (later calls
                             return HCOV_ESTATE; destroy it).  Ignored with
                             fixed_rank > 0. */
} hcov_opts;

#define HCOV_ADM_MIN 0
#define HCOV_ADM_MAX 1
#define HCOV_ADM_WEAK 2

#define HCOV_QUAD_DIRECT 0
#define HCOV_QUAD_PCG 1

#define HCOV_SAT_RETRY 0
#define HCOV_SAT_ERROR 1

/* Structure and work counters of a context (see hcov_stats). */
typedef struct {
  int64_t n;
  int leaf;
  int depth;                  /* cluster-tree depth D (2^D leaves) */
  int64_t n_dense_blocks;
  int64_t n_lr_blocks;
  int64_t dense_entries;      /* stored entries of dense blocks */
  int64_t lr_rows;            /* sum over low-rank blocks of (rows + cols) */
  int max_rank_seen;          /* largest rank after the last assembly/factorisation */
  double mean_rank;
  int64_t bytes_device;       /* device memory held by the context */
  int64_t bytes_factor;       /* bytes of the stored factor (actual ranks) */
  double ms_tree, ms_assemble, ms_factor, ms_solve;   /* last phase times */
  int64_t n_steps;            /* sweep steps of the factorisation (= 2^D) */
  int64_t n_launches_factor;  /* kernel launches of one factorisation */
  int64_t n_graph_replays;    /* factorisations run as a replay of the captured sweep */
  int64_t n_sketch_retries;   /* factorisations redone with wider sketches */
  int sketch_saturated;       /* saturated sketches in the last factorisation */
  double mean_sketch_width;   /* mean sketch width of the low-rank blocks */
  int pcg_iters;              /* PCG iterations of the last quadratic form */
  double pcg_relres;          /* its final ||z - C~ x|| / ||z|| */
  int64_t n_gemm_grouped;     /* GEMM launches of one factorisation on the
                                 two-group kernel */
  int64_t n_autotune_switched;/* GEMM launches the autotuning moved to the
                                 other kernel (0 before / without it) */
  double gemm_flops_factor;   /* algorithmic GEMM flops of one factorisation
                                 at the current ranks (2 m n k per product) */
  double gemm_bytes_factor;   /* its algorithmic GEMM bytes (operands read
                                 once, outputs written, accumulations read) */
  int64_t n_replans;          /* plan rebuilds that grew block capacities
                                 (opts.initial_rank_cap) */
  int64_t bytes_lowrank;      /* bytes of the U and V arenas of the low-rank
                                 blocks at their current capacities */
} hcov_stats_t;

typedef struct hcov_ctx hcov_ctx;

/* Fill *o with the defaults listed above. */
void hcov_opts_default(hcov_opts* o);

/* hcov_build -- cluster tree, block cluster tree and H-matrix assembly.
 *
 * Defines the problem of [HLIBCov Sec. 1]: n locations s_i in R^2 and the
 * Matérn covariance of Eq. (3).  Builds on the GPU
 *   - the cluster tree: recursive bisection of the index set into two
 *     equal-sized subsets [HLIBCov Sec. 2.2] by an axis-parallel cut across
 *     the longer side of each cluster's bounding box, down to leaves of at
 *     most `leaf` points (n_min of Sec. 2.2);
 *   - the block cluster tree with standard admissibility Adm_eta
 *     [HLIBCov Appendix A, Eq. (stand_cond)];
 *   - the H-matrix C~(theta): dense leaves exactly, admissible leaves by ACA
 *     followed by SVD recompression to ||M - M~|| <= eps ||M||
 *     [HLIBCov Sec. 2.2 and Appendix B remark].
 *
 * locs_xy : host pointer, n x 2 doubles, row major (x0, y0, x1, y1, ...);
 *           copied; must be finite.
 * n       : number of locations, >= 1.
 * theta   : see hcov_theta; sigma2, ell, nu > 0, nugget >= 0.
 * eps     : block accuracy in (0, 1).
 * leaf    : leaf size in [2, 128].
 * eta     : admissibility parameter > 0.
 * opts    : NULL for defaults.
 * hip_stream : hipStream_t to order all work on (NULL = default stream).
 * out     : receives the new context (NULL on error).
 */
int hcov_build(const double* locs_xy, int64_t n, hcov_theta theta, double eps,
               int leaf, double eta, const hcov_opts* opts, void* hip_stream,
               hcov_ctx** out);

/* Re-assemble C~ for new parameters, reusing both trees [HLIBCov Appendix B:
 * every likelihood evaluation rebuilds the matrix for its theta].  Invalidates
 * the factor. */
int hcov_set_theta(hcov_ctx* ctx, hcov_theta theta);

/* H-Cholesky C~ = L~ L~^T in place [HLIBCov Eq. (2), Sec. 2.2: H-matrix
 * factorisation with the same fixed accuracy eps for the factor].
 *
 * Returns HCOV_ENOTSPD if a diagonal leaf has a non-finite pivot or a pivot
 * that does not exceed 64 p u times its diagonal entry (leaf order p,
 * u = 2^-53): Sec. 3 notes that nearly dependent columns (coincident
 * locations) break the factorisation and that a nugget (Sec. 5.2) cures it.
 *
 * Every updated low-rank block is recompressed to accuracy eps from a
 * randomised sketch (width: see opts.oversample).  When a block keeps a rank
 * of at least the width minus one while the sketch is narrower than the
 * block, the sketch is saturated and eps is no longer guaranteed for that
 * block.  After such a factorisation every block's rank hint becomes the
 * rank it kept, its sketch width plus max(8, width / 4) where the sketch
 * saturated.  With
 * HCOV_SAT_RETRY the matrix is re-assembled and the factorisation redone
 * with the new widths, up to 4 times; a sketch saturated at the widest width
 * (the block's room + 16), saturation after the last retry, or any
 * saturation with HCOV_SAT_ERROR returns HCOV_ERANK.  The factorisation is
 * never reported as done (HCOV_OK) with a saturated sketch.  The hints
 * persist in the context and change only after a saturated factorisation:
 * later factorisations (new theta) start from them, and repeating an
 * evaluation gives the same bits.
 *
 * A block whose kept rank exceeds its room (max_rank, or the grown room of
 * opts.initial_rank_cap) returns HCOV_ERANK when the room is max_rank;
 * below it the rooms grow, the plan and buffers are rebuilt and the
 * assembly and factorisation repeat inside this call (at most 8 rebuilds per
 * call).  Device pointers into the context's buffers are not exposed, so a
 * rebuild is invisible to the caller except in time and memory. */
int hcov_cholesky(hcov_ctx* ctx);

/* log|C~| = 2 sum_i log L~_ii [HLIBCov Eq. (2)], FP64 reduction in a fixed
 * order.  Requires hcov_cholesky (else HCOV_ESTATE). */
int hcov_logdet(hcov_ctx* ctx, double* out_logdet);

/* x = (L~ L~^T)^{-1} z: forward solve L~ v = z [HLIBCov Eq. (2)] then the
 * backward solve L~^T x = v.  z and x hold n doubles in external order, both
 * on the host or both on the device (`where`).  Requires hcov_cholesky. */
int hcov_solve(hcov_ctx* ctx, const double* z, double* x, int where);

/* Forward solve only: v = L~^{-1} P z (v in cluster order) and
 * quad = v^T v.  v may be NULL. */
int hcov_forward(hcov_ctx* ctx, const double* z, double* v, double* quad, int where);

/* y = P^T L~ xi: sample a field with covariance L~ L~^T from a standard
 * normal xi given in cluster order [HLIBCov Sec. 5.1 generates Z0 = L~ xi].
 * Result in external order.  Requires hcov_cholesky. */
int hcov_sample(hcov_ctx* ctx, const double* xi, double* y, int where);

/* y = C~ x (H-matrix times vector, [HLIBCov Table 1 "C~ z"]), external order.
 * Requires an assembled, not yet factorised context, or opts.keep_matrix
 * (else HCOV_ESTATE). */
int hcov_matvec(hcov_ctx* ctx, const double* x, double* y, int where);

/* y = L~ L~^T x (the factorised matrix times a vector, external order;
 * the factor's product with a vector of [HLIBCov Table 1]).  Requires
 * hcov_cholesky and opts.keep_matrix (for the vector workspace). */
int hcov_factor_matvec(hcov_ctx* ctx, const double* x, double* y, int where);

/* Accuracy of the factorisation by power iteration [HLIBCov Sec. 3, the error
 * columns of Tables 2, 3 and 5], each from its own seeded Gaussian start
 * vector and `iters` iterations (each estimate is a lower bound that
 * increases towards the norm):
 *   norm_c   = ||C~||_2,
 *   err_fact = ||C~ - L~ L~^T||_2,
 *   err_inv  = ||I - (L~ L~^T)^{-1} C~||_2 (power iteration on A^T A).
 * Requires a factorised context built with opts.keep_matrix.  Any output
 * pointer may be NULL. */
int hcov_error_norms(hcov_ctx* ctx, int iters, uint64_t seed, double* norm_c, double* err_fact,
                     double* err_inv);

/* y = C x with the exact entries of Eq. (3) evaluated on the fly on the
 * device (O(n^2) Matérn evaluations, no storage), external order: the
 * reference the H-matrix approximates. */
int hcov_exact_matvec(hcov_ctx* ctx, const double* x, double* y, int where);

/* Approximation errors against the exact C of Eq. (3) by power iteration
 * with exact products (hcov_exact_matvec), as the error columns of
 * [HLIBCov Tables 2 and 3]:
 *   err_c    = ||C - C~||_2,
 *   err_cinv = ||C (L~ L~^T)^{-1} - I||_2 (the factor's inverse standing for
 *              C~^{-1}; power iteration on B^T B).
 * Requires a factorised context built with opts.keep_matrix. */
int hcov_exact_norms(hcov_ctx* ctx, int iters, uint64_t seed, double* err_c, double* err_cinv);

/* H-log-likelihood of Eq. (2) [HLIBCov Sec. 1]:
 *   L~ = -n/2 log(2 pi) - sum_i log L~_ii - 1/2 v^T v,  L~ v = z,
 * returned with the paper's sign (+L; the listing of Appendix B returns -L
 * for minimisation).  Runs hcov_cholesky when the factor is not current.
 * out_logdet (log|C~|) and out_quad (z^T C~^{-1} z) may be NULL. */
int hcov_loglik(hcov_ctx* ctx, const double* z, int where, double* out_ll,
                double* out_logdet, double* out_quad);

/* Structure, memory and per-phase time counters. */
int hcov_stats(const hcov_ctx* ctx, hcov_stats_t* out);

/* Conservative device-memory bound of hcov_build + hcov_cholesky for n
 * points at this leaf size and rank capacity, from sizes alone (no tree is
 * built): dense near-field leaves ~ 16 n leaf, low-rank factors
 * ~ 24 n (D+1) max_rank, plus scratch.  Used for admission control in
 * serving; the exact figure after a build is hcov_stats().bytes_device. */
int hcov_estimate_bytes(const double* locs_xy, int64_t n, double eps, int leaf,
                        double eta, const hcov_opts* opts, size_t* out_bytes);

/* Cluster permutation: perm[i] = external index of cluster-order position i. */
int hcov_perm(const hcov_ctx* ctx, int64_t* perm);

void hcov_destroy(hcov_ctx* ctx);

/* ------------------------------------------------------------ outer loop */

/* Objective of the simplex minimiser: f(x[0..dim)) for `user`. */
typedef double (*hcov_objective_fn)(const double* x, int dim, void* user);

/* Nelder-Mead minimisation (Nelder & Mead 1965; the paper's optimiser is a
 * derivative-free simplex search, Sec. 5 and the driver of Appendix B):
 * reflection 1, expansion 2, contraction 1/2, shrink 1/2, initial simplex
 * x0 and x0 + steps[k] e_k, stable ordering of the vertices.  Stops when the
 * largest vertex distance to the centroid is below size_tol or after
 * max_evals evaluations.  hist_x (max_evals x dim) and hist_f (max_evals)
 * receive every evaluation in order when not NULL.  Host only. */
int hcov_nm_minimize(hcov_objective_fn f, void* user, const double* x0, const double* steps, int dim,
                     int max_evals, double size_tol, double* out_x, double* out_f, int* out_evals,
                     double* hist_x, double* hist_f);

/* Maximum-likelihood fit of theta = (sigma^2, ell, nu) [Sec. 5]: minimises
 * -L~ of Eq. (2) with hcov_nm_minimize, each evaluation re-assembling C~ for
 * its theta on the context's trees (hcov_set_theta + hcov_loglik).  Points
 * outside the domain (or not positive definite) count as +inf.  steps: NULL
 * for (0.01, 0.04, 0.02), the paper's initial steps reordered to
 * (sigma^2, ell, nu).  hist_theta (max_evals x 3), hist_negll (max_evals)
 * optional. */
int hcov_fit(hcov_ctx* ctx, const double* z, int where, const double* theta0, const double* steps,
             double nugget, int max_evals, double size_tol, double* out_theta, double* out_ll, int* out_evals,
             double* hist_theta, double* hist_negll);

/* Kernel timing: between hcov_profile_begin(ctx, kind) and
 * hcov_profile_end, every launch of the given stage kind (0 grouped GEMM,
 * by either GEMM kernel, 1 TSQR segment, 2 TSQR reduce, 3 small SVD / pivoted QR, 4 diagonal leaf
 * potrf, 5 triangular solve, 9 multiplication by a stored leaf inverse) is
 * bracketed by HIP events on the stream it runs on.  hcov_profile_end
 * synchronises and returns the launch count, the summed event time (ms),
 * the algorithmic FP64 flops of those launches (GEMM: 2 m n k per product;
 * potrf: p^3/3; solve and multiplication: p^2 per column; 0 for the other
 * kinds) and their algorithmic bytes (every operand read once, every output
 * written once and read once more when accumulated: GEMM 8 (m k + k n) per
 * product plus 8 m n or 16 m n per job, 4-byte elements in FP32 jobs;
 * potrf 16 p^2; solve and multiplication 8 p (p + 2 columns)).  Any output
 * pointer may be NULL.  Other values of kind are EINVAL. */
int hcov_profile_begin(hcov_ctx* ctx, int stage_kind);
int hcov_profile_end(hcov_ctx* ctx, int64_t* launches, double* total_ms, double* flops, double* bytes);
/* The per-launch durations (ms, launch order) of the last profiling session:
 * up to max_n values into times_ms (may be NULL), the count into *n_out. */
int hcov_profile_times(const hcov_ctx* ctx, double* times_ms, int64_t max_n, int64_t* n_out);

/* Eq. (3) on the device for n given distances h (host arrays): test access to
 * the device Matérn / K_nu evaluation used by the assembly. */
int hcov_matern_eval(hcov_theta theta, const double* h, double* out, int64_t n);

/* hcov_matern_eval without allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture elsewhere in the process, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments and result
 * as hcov_matern_eval (host arrays h, out of n doubles), on the current
 * device and its null stream.  The device staging of h and out lives in a
 * fixed array of HCOV_NOALLOC_MAX_N x 2 doubles (4 MiB) that each GPU holds
 * for the life of the process; n > HCOV_NOALLOC_MAX_N returns HCOV_EINVAL
 * before any device work.  Calls on one GPU share that array: calls from
 * threads of this process are serialised by a per-device lock, calls that
 * overlap from other code paths on the same array race. */
#define HCOV_NOALLOC_MAX_N 262144
int hcov_matern_eval_noalloc(hcov_theta theta, const double* h, double* out, int64_t n);

const char* hcov_strerror(int code);
const char* hcov_last_error(const hcov_ctx* ctx);

/* ------------------------------------------------------------ tree access
 * Structural output for bit-exact checks against the reference trees. */

/* Depth D and the number of block-tree leaves. */
int hcov_tree_sizes(const hcov_ctx* ctx, int* depth, int64_t* n_blocks);
/* bbox: (2^(D+1)-1) x 4 doubles (xmin,xmax,ymin,ymax) in level order
 * (level l node i at index 2^l-1+i); blocks: n_blocks x 4 int64 rows
 * (level, row node, column node, kind) with kind 1 = low rank, 0 = dense, in
 * breadth-first order. */
int hcov_tree_dump(const hcov_ctx* ctx, double* bbox, int64_t* blocks);

/* ------------------------------------------------------------ serving
 * A request loop for many likelihood evaluations of different n and theta
 * (an optimiser re-evaluating one data set, or independent data sets).  The
 * server owns `slots` worker threads, each with its own HIP stream, so that
 * up to `slots` evaluations run concurrently and their kernels overlap on
 * the GPU.  Requests are admitted in arrival order as soon as a slot is free
 * and the estimate of their device memory (hcov_estimate_bytes) fits in the
 * remaining budget; a request larger than the whole budget runs alone.
 * Every evaluation is the same computation as hcov_build + hcov_loglik on
 * its own context, so its result does not depend on the other requests.
 *
 * Data sets registered with hcov_server_dataset stay resident (trees, plan
 * and factor storage), and requests naming them only re-assemble and
 * re-factorise for the new theta [HLIBCov Sec. 4: the likelihood is
 * maximised over theta for fixed locations]; their memory is charged to the
 * budget until hcov_server_release.  Requests on one data set run one at a
 * time in arrival order.
 *
 * All server calls are thread safe.  The server must be destroyed before the
 * process exits; hcov_server_destroy waits for the admitted requests and
 * drops the queued ones. */
typedef struct hcov_server hcov_server;

typedef struct {
  const double* locs;   /* host n x 2 locations (copied at submit); NULL
                           when `dataset` names a resident data set */
  int64_t n;            /* number of locations (= the data set's n) */
  const double* z;      /* host observations, external order (copied) */
  hcov_theta theta;
  double eps;           /* used only without a data set */
  int leaf;
  double eta;
  int dataset;          /* 0, or an id from hcov_server_dataset */
} hcov_request;

typedef struct {
  int status;           /* HCOV_OK or the evaluation's error code */
  double loglik, logdet, quad;   /* as hcov_loglik */
  double queue_ms;      /* submit -> admission */
  double service_ms;    /* admission -> completion */
  double latency_ms;    /* submit -> completion */
} hcov_result;

/* slots in [1, 64]; mem_budget_bytes = 0: 90% of the device memory free at
 * creation; opts: build options of every context (NULL = defaults; the
 * allocator fields are replaced by stream-ordered allocation). */
int hcov_server_create(int slots, size_t mem_budget_bytes, const hcov_opts* opts, hcov_server** out);
/* Registers a resident data set (built now, on its own stream). */
int hcov_server_dataset(hcov_server* s, const double* locs, int64_t n, hcov_theta theta, double eps, int leaf,
                        double eta, int* id);
/* Frees a data set once its queued requests have run. */
int hcov_server_release(hcov_server* s, int id);
/* Queues a request; *ticket identifies its result. */
int hcov_server_submit(hcov_server* s, const hcov_request* req, uint64_t* ticket);
/* HCOV_OK and *out filled when done (the result is then forgotten),
 * HCOV_EAGAIN while queued or running, HCOV_EINVAL for unknown tickets. */
int hcov_server_poll(hcov_server* s, uint64_t ticket, hcov_result* out);
/* Blocks until the request is done, then as hcov_server_poll. */
int hcov_server_wait(hcov_server* s, uint64_t ticket, hcov_result* out);
void hcov_server_destroy(hcov_server* s);

#ifdef __cplusplus
}
#endif
#endif /* HCOV_H_ */
