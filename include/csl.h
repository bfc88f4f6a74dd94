/*
 * csl.h -- C ABI of the MI355X (gfx950) solver for complex-shifted
 * Laplacian systems with the absolute-value preconditioner of
 * Lin, Li & Hon, "Absolute-value based preconditioner for complex-shifted
 * Laplacian systems" (arXiv:2408.00488).
 *
 * Problem (Section 1, Eq. (1)):  (K + lambda I) z = f,  lambda = alpha + i beta,
 * K the 5-point (2-D) or 7-point (3-D) finite-difference matrix of
 * -div(a grad) on a uniform grid of a rectangular domain, homogeneous
 * Dirichlet boundary.  Face coefficients are harmonic means of the nodal
 * samples of a; a face on the boundary carries the adjacent nodal value.
 *
 * Solver: preconditioned MINRES on the real symmetric 2x2 block form
 * (Eq. (2), read as A = [[K + alpha I, beta I], [beta I, -(K + alpha I)]]
 * acting on [Re z; -Im z]) with the preconditioner
 * P = blkdiag(sqrt((abar L + alpha I)^2 + beta^2 I)) twice (Eq. (4)),
 * applied through multi-axis sine transforms (Section 2.3).
 *
 * Data layout.  Every vector is a DEVICE array of M = n_0 * ... * n_{d-1}
 * complex numbers stored as interleaved (re, im) double pairs, indexed by
 * interior grid node in C order (last axis contiguous).  The real block
 * vector [x1; x2] is stored as x1 + i x2.  The nodal coefficient is a DEVICE
 * array of M doubles in the same order.  Grid axis k has n[k] interior
 * points, mesh width h_k = length[k] / (n[k] + 1), 3 <= n[k] <= 1023.  With
 * n[k] + 1 a power of two the sine transform along the axis runs as the LDS
 * FFT or the dense sine matrix; any other n[k] takes the dense sine matrix
 * on the matrix cores only, whose cost grows as n[k]^2 per line.
 *
 * Ownership.  The caller owns every vector and coefficient buffer and keeps
 * it alive while work that uses it is queued.  A problem handle owns a copy
 * of the coefficient, the per-axis eigenvalue tables and all workspaces,
 * allocated in create_problem and freed in destroy_problem; solves allocate
 * nothing.  A problem (and a batch) may be used by one solve at a time.
 *
 * Streams.  Every call takes a hipStream_t (0 = default stream) and orders
 * its device work on it.  Calls that return a solve info (info != NULL)
 * synchronise that stream before returning.
 *
 * Errors.  Every entry point returns a csl_status and never aborts;
 * csl_last_error() returns a thread-local message for the last non-OK
 * status.  Non-convergence is a status: the output holds the last iterate
 * and the info records iterations and residuals.
 */
#ifndef CSL_H
#define CSL_H

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum csl_status {
    CSL_OK = 0,
    CSL_ERR_ARG = 1,            /* invalid argument (message says which)        */
    CSL_ERR_SINGULAR = 2,       /* preconditioner singular: beta = 0 and
                                   abar*mu_k + alpha = 0 for some mode k        */
    CSL_ERR_NOT_CONVERGED = 3,  /* maxit reached; output = last iterate          */
    CSL_ERR_BREAKDOWN = 4,      /* <z, v> < 0 in the Lanczos process
                                   (preconditioner not positive definite)       */
    CSL_ERR_NONFINITE = 5,      /* NaN / Inf in the data or the recurrences     */
    CSL_ERR_HIP = 6,            /* a HIP runtime call failed                     */
    CSL_ERR_OOM = 7,            /* device allocation failed                      */
    CSL_ERR_TIMEOUT = 8         /* the solver kernel exceeded its time limit     */
} csl_status;

typedef struct csl_problem_s *csl_problem;
typedef struct csl_batch_s *csl_batch;
typedef struct csl_paradiag_s *csl_paradiag;

/* Grid of the rectangular domain (Section 1): dim in {2, 3}; n[k] interior
 * points along axis k (axis dim-1 contiguous); length[k] > 0 the side
 * length (a value <= 0 means 1).  Unused entries are ignored. */
typedef struct csl_grid {
    int dim;
    int n[3];
    double length[3];
} csl_grid;

/* How abar of K_bar = abar L is chosen (Eq. (4) uses sqrt(a_min a_max)). */
enum {
    CSL_ABAR_MEAN = 0,      /* arithmetic mean of the nodal samples (default) */
    CSL_ABAR_GEOMEAN = 1,   /* sqrt(min c_e * max c_e) over face coefficients  */
    CSL_ABAR_GIVEN = 2      /* csl_problem_opts.abar                            */
};

/* Arithmetic of the preconditioner's sine transforms and mode scaling. */
enum {
    CSL_PREC_FP64 = 0,      /* everything FP64                                  */
    CSL_PREC_FP32 = 1       /* transforms and scaling in FP32; Lanczos vectors,
                               inner products, norms and rotations stay FP64   */
};

/* How the orthonormal DST-I along an axis is computed (the W of
 * P^{-1} = W diag(s) W, Section 2.3).  All give the same transform up to
 * rounding. */
enum {
    CSL_DST_AUTO = 0,       /* per axis, the faster of FFT and GEMM, timed on
                               this device the first time a grid shape and
                               precision is seen in the process (GEMM on
                               every axis with n + 1 not a power of two)   */
    CSL_DST_FFT = 1,        /* FFT of the odd extension, staged in LDS
                               (CSL_ERR_ARG if an axis has n + 1 not a
                               power of two)                               */
    CSL_DST_GEMM = 2,       /* product with the dense n x n sine matrix on
                               the matrix cores, for axes with
                               15 <= n <= 127 or n + 1 not a power of two
                               (any n up to 1022); FFT on the other axes   */
    CSL_DST_GEMM16 = 3      /* the same axes as CSL_DST_GEMM, with the
                               preconditioner's products on FP16 matrix
                               cores: every line scaled by a power of two,
                               matrix and line split into FP16 high and low
                               parts, three products accumulated in FP32
                               (FP32 accuracy).  Needs CSL_PREC_FP32; the
                               FP64 pass of the Lanczos vectors keeps the
                               FP64 product                                */
};

typedef struct csl_problem_opts {
    int abar_rule;          /* CSL_ABAR_*                                       */
    int pinv_prec;          /* CSL_PREC_*                                       */
    double abar;            /* used when abar_rule == CSL_ABAR_GIVEN            */
    int tile_elems;         /* target LDS elements per sine-transform tile of
                               the contiguous axis (0 = default: 2048 FP64,
                               4096 FP32); larger tiles mean fewer phase
                               hand-offs, smaller ones more parallelism       */
    int dst_engine;         /* CSL_DST_*                                        */
    int reserved[2];
} csl_problem_opts;

typedef struct csl_solve_opts {
    double tol;             /* relative tolerance (default 1e-8 when <= 0)      */
    int maxit;              /* iteration limit (default 1000 when <= 0)         */
    int check_true_residual;/* 1: also require ||f - (K+lambda I) z|| / ||f||
                               <= tol once the recurrence estimate passed      */
    int timeout_ms;         /* kernel time limit (default 60000 when <= 0): past
                               it no further phase is started, the launch
                               returns within one phase and an unfinished
                               solve reports CSL_ERR_TIMEOUT                */
    int reserved[3];
} csl_solve_opts;

typedef struct csl_solve_info {
    int status;             /* csl_status of this system                        */
    int iters;              /* MINRES iterations (one A and one P^{-1} each)    */
    double relres_est;      /* |eta_k| / |eta_0|: P^{-1}-norm residual ratio     */
    double relres_true;     /* ||f - (K + lambda I) z||_2 / ||f||_2             */
} csl_solve_info;

/* Create a problem: copies a (device, M doubles, all finite and > 0),
 * computes the face-coefficient bounds and abar, the per-axis eigenvalues
 * mu_k = (4/h^2) sin^2(k pi / (2(n+1))) of L (Section 2.3), checks that P is
 * nonsingular, and allocates the workspaces.  Synchronises `s`.
 * opts may be NULL (defaults: mean rule, FP64). */
csl_status create_problem(const csl_grid *grid, const double *a_nodal,
                          double alpha, double beta,
                          const csl_problem_opts *opts, hipStream_t s,
                          csl_problem *out);

csl_status destroy_problem(csl_problem p);

/* A second problem with p's grid, coefficient (copied from p's own copy),
 * shift, abar, precision, sine-transform engines and schedule, and
 * workspaces of its own, without timing the engines again: several
 * right-hand sides of one shifted system are then solved together by
 * batching p and its clones.  Synchronises s. */
csl_status problem_clone(csl_problem p, hipStream_t s, csl_problem *out);

/* Query: abar used by P, and the face-coefficient bounds a_min, a_max
 * (Lemma 3).  Any pointer may be NULL. */
csl_status problem_info(csl_problem p, double *abar, double *a_min,
                        double *a_max);

/* Schedule of the problem's own solves (minres_solve, minres_adjoint):
 * tile_points grid points per scheduling tile (0 = about one tile per
 * workgroup and phase, which lets a single solve fill the device; 1 = one
 * LDS chunk per tile), the LDS line budget (0 or 32768 = default, 65536
 * = 64 KiB) and the workgroup size of the persistent solver, block_threads:
 * 0 = 512 where allowed, else 256; 256; 512, which is allowed for problems
 * whose sine transforms all run on the FFT (CSL_ERR_ARG otherwise); or 1024,
 * the plane phase, for 3-D problems with the FFT on every axis and n0, n1
 * <= 127 (CSL_ERR_ARG otherwise): one workgroup per CU holds the real or
 * the imaginary part of a plane of axes 0 and 1 in LDS and applies the
 * transforms of P^{-1} along both of them (Section 2.3) in one phase; its
 * workgroups have 1024 threads with the FP32 preconditioner and 512 with
 * the FP64 one, whose FP64 plane leaves LDS for eight waves' line buffers
 * only; tile_points and lds_bytes then apply to the contiguous-axis phases;
 * tile_elems, the LDS elements of a chunk (0 = the creation-time tiling;
 * chunks smaller than that are accepted while every tile keeps a partial-sum
 * slot, on grids of at most 65536 points down to 512 elements; CSL_ERR_ARG
 * otherwise, the previous schedule staying in force).  Batches keep their
 * own schedule.  Synchronises s. */
csl_status problem_set_schedule(csl_problem p, int tile_points, int lds_bytes,
                                int block_threads, int tile_elems, hipStream_t s);

/* Lanczos coefficients of the problem's last completed solve (its own
 * minres_solve / minres_adjoint, or its system within a batch_solve):
 * delta_1..delta_k, the diagonal of the tridiagonal T_k that MINRES builds
 * for P^{-1} A (Section 2.2), and gamma_2..gamma_{k+1}, its off-diagonal
 * (gamma_{k+1} couples step k to the next), k = the steps taken (at most
 * 4096 recorded).  delta, gamma: host arrays of cap entries (the first
 * min(cap, k) are written; may be NULL when cap = 0); *count = k.
 * Synchronises s: call it on the stream of the solve. */
csl_status problem_lanczos(csl_problem p, double *delta, double *gamma, int cap,
                           int *count, hipStream_t s);

/* Ritz values of P^{-1} A from the last completed solve: the eigenvalues of
 * T_k, ascending (host bisection on Sturm counts, O(k^2) work).  Their
 * extremes approach the extreme eigenvalues that Theorem 3 bounds; all of
 * them lie between the smallest and largest eigenvalue.  theta: host array
 * of cap entries; *count = k.  Synchronises s. */
csl_status problem_ritz(csl_problem p, double *theta, int cap, int *count, hipStream_t s);

/* Host utility (no device work): the eigenvalues of the symmetric
 * tridiagonal matrix with diagonal d[0..k-1] and off-diagonal e[0..k-2],
 * ascending, into theta[0..k-1] (host arrays), by the bisection that
 * problem_ritz uses.  k >= 0; pointers may be NULL when k = 0. */
csl_status csl_tridiagonal_eigenvalues(const double *d, const double *e, int k, double *theta);

/* Sine-transform engine in use along each axis (CSL_DST_FFT, CSL_DST_GEMM or
 * CSL_DST_GEMM16; entries past the grid's dimension are CSL_DST_FFT). */
csl_status problem_dst_engines(csl_problem p, int engines[3]);

/* y = A x for the block matrix of Eq. (2); in complex storage
 * y = (K + lambda I) conj(x).  x, y: device, M complex; must not alias. */
csl_status apply_A(csl_problem p, const double *x, double *y, hipStream_t s);

/* y = P^{-1} x with P of Eq. (4) (the same real operator on Re and Im),
 * through forward sine transforms along every axis, the per-mode factor
 * 1/sqrt((abar mu + alpha)^2 + beta^2) and inverse transforms
 * (Section 2.3).  x, y: device, M complex; may alias. */
csl_status apply_Pinv(csl_problem p, const double *x, double *y,
                      hipStream_t s);

/* Solve (K + lambda I) z = f by preconditioned MINRES on the block system
 * from z0 = 0 (Section 3).  f, z: device, M complex, must not alias.
 * Stops after iteration k when |eta_k|/|eta_0| <= tol and (if requested)
 * the true relative residual <= tol.  One persistent kernel launch.
 * If info != NULL, synchronises `s`, fills info and returns its status;
 * otherwise returns CSL_OK once the work is queued. */
csl_status minres_solve(csl_problem p, const double *f, double *z,
                        const csl_solve_opts *opts, csl_solve_info *info,
                        hipStream_t s);

/* minres_solve for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * problem is given directly (grid, a_nodal, alpha, beta, opts as for
 * create_problem; a_nodal is read in place, not copied) and solved once,
 * with no handle and no allocation.  Every workspace of the solve lives in
 * one static device array of 64 MiB per GPU that the library holds from the
 * moment it is loaded until the process ends.  Limits: every axis needs
 * n + 1 a power of two (the FFT engine; dst_engine AUTO or FFT), and the
 * grid's workspace must fit the 64 MiB (2-D grids up to 511 x 511, 3-D up to
 * 63^3 in FP64): larger grids, or an axis without an FFT, return CSL_ERR_ARG
 * before any device work.  Set-up runs on every call and synchronises s once
 * (the coefficient check and abar, as in create_problem); the solve itself
 * is minres_solve's kernel, and with info != NULL s is synchronised again.
 * All calls on one GPU share its array: calls that overlap on one device
 * (from several threads or streams) race and give undefined results; one
 * call's device work must complete before the next call on that device is
 * queued on another stream.  f, z: device, M complex, must not alias. */
csl_status minres_solve_noalloc(const csl_grid *grid, const double *a_nodal, double alpha,
                                double beta, const csl_problem_opts *opts, const double *f,
                                double *z, const csl_solve_opts *sopts, csl_solve_info *info,
                                hipStream_t s);

/* Adjoint of z = (K + lambda I)^{-1} f for a real loss L(z).
 * gz = dL/dRe z + i dL/dIm z (device, M complex).  One extra MINRES solve
 * y = (K + conj(lambda) I)^{-1} gz on the same symmetric block matrix, then
 *   gf = y (device, M complex, written),
 *   *galpha = -Re(y^H z), *gbeta = Im(y^H z) (device doubles, written),
 *   ga[p] += sum over faces e of p of dL/dc_e * dc_e/da_p (device, M
 *   doubles, ACCUMULATED), dL/dc_e = -Re(y^H dK/dc_e z).
 * z is the forward solution (device, M complex).  The dependence of abar
 * on a is ignored (P does not change the exact solution).  Any of gf,
 * galpha, gbeta, ga may be NULL.  Synchronises `s` when info != NULL. */
csl_status minres_adjoint(csl_problem p, const double *z, const double *gz,
                          double *gf, double *galpha, double *gbeta,
                          double *ga, const csl_solve_opts *opts,
                          csl_solve_info *info, hipStream_t s);

typedef struct csl_batch_opts {
    double tol;
    int maxit;
    int check_true_residual;
    int timeout_ms;
    int grid_size;          /* workgroups of the persistent launch; 0 = auto   */
    int use_graph;          /* 1: replay a captured hipGraph per solve          */
    int tile_points;        /* grid points per scheduling tile (0 = 8192);
                               larger tiles mean fewer cross-workgroup
                               hand-offs, smaller ones more parallelism    */
    int lds_bytes;          /* LDS line budget per workgroup: 0 = per
                               problem (32 KiB unless lines of 2048 need
                               64), 65536 = 64 KiB for every problem (twice
                               the lines per strided tile); 32768 = 0      */
    int block_threads;      /* workgroup size of the persistent solver: 0 =
                               512 if every problem allows it (the FFT on
                               every axis), else 256; 256; 512 (CSL_ERR_ARG
                               unless every problem allows it); 1024, the
                               plane phase (CSL_ERR_ARG unless every problem
                               is 3-D with the FFT on every axis and n0, n1
                               <= 127, all with one preconditioner
                               precision)                                  */
} csl_batch_opts;

/* Schedule chosen by batch_tune or problem_tune, or in use
 * (problem_schedule, batch_schedule: candidates = 0, ms = ms_default = 0). */
typedef struct csl_batch_tuning {
    int tile_points;        /* chosen grid points per tile                      */
    int lds_bytes;          /* chosen LDS budget (32768 or 65536)               */
    int grid_size;          /* workgroups of the persistent launch              */
    int candidates;         /* schedules timed                                  */
    double ms;              /* time of one solve with the chosen schedule       */
    double ms_default;      /* time with the creation-time schedule             */
    int block_threads;      /* workgroup size of the persistent solver          */
    int tile_elems;         /* chunk size (LDS elements) of a problem's own
                               solves, 0 = the creation-time tiling (always 0
                               for batches, which keep that tiling)        */
} csl_batch_tuning;

/* Group `count` problems (any grids, shifts and precisions) into one
 * persistent launch: every workgroup takes tiles from whichever system has
 * work ready, so systems of uneven size share the device.  The problems
 * must outlive the batch and must not be solved separately while a batch
 * solve is queued.  opts may be NULL. */
csl_status batch_create(const csl_problem *problems, int count,
                        const csl_batch_opts *opts, csl_batch *out);

/* Solve every system of the batch: f[j], z[j] are device pointers for
 * system j (host arrays of `count` pointers).  The z[j] are distinct and
 * none is any f[i] (CSL_ERR_ARG otherwise).  One (graph) launch.  If
 * infos != NULL (host array of `count`), synchronises `s`, fills the infos
 * and returns CSL_OK only if every system converged (else the first
 * non-OK status).  At the time limit, systems already finished keep their
 * status and solution; the others report CSL_ERR_TIMEOUT. */
csl_status batch_solve(csl_batch b, const double *const *f, double *const *z,
                       csl_solve_info *infos, hipStream_t s);

/* Adjoint of every system of the batch at once (minres_adjoint for each
 * system j, derived from Eq. (1)): z[j] the forward solution and gz[j] =
 * dL/dRe z_j + i dL/dIm z_j (device, M_j complex each; host arrays of
 * `count` pointers).  The adjoint solves y_j = (K + conj(lambda_j) I)^{-1}
 * gz[j] of all systems run in one persistent launch (the batch's schedule),
 * then, system by system in order:
 *   gf[j] = y_j (device, M_j complex, written; gf or any gf[j] may be NULL),
 *   galpha[j] = -Re(y_j^H z_j), gbeta[j] = Im(y_j^H z_j) (device arrays of
 *   `count` doubles, written; either may be NULL),
 *   ga[p] += sum over the systems of dL_j/da_p (device, M doubles,
 *   ACCUMULATED in the order j = 0, 1, ...: the gradient of a loss summed
 *   over systems that share one coefficient; every system must then be on
 *   one grid, else CSL_ERR_ARG; may be NULL).
 * opts: tolerance and limits of the adjoint solves (NULL: the batch's).
 * Uses each problem's own adjoint workspaces: no problem of the batch may be
 * solved or adjoint-solved elsewhere while this is queued.  If infos != NULL
 * (host array of `count`), synchronises s, fills them (the adjoint solves)
 * and returns CSL_OK only if every system converged. */
csl_status batch_adjoint(csl_batch b, const double *const *z, const double *const *gz,
                         double *const *gf, double *galpha, double *gbeta, double *ga,
                         const csl_solve_opts *opts, csl_solve_info *infos, hipStream_t s);

/* Autotuner of a problem's own schedule: solves (K + lambda I) z = f with
 * each candidate tile size, LDS budget and allowed workgroup size, and on
 * grids of at most 65536 points also chunks of 512 and 1024 elements (tol
 * 1e-8), timing each on stream s, and keeps the fastest
 * (problem_set_schedule).  With dst_engine CSL_DST_AUTO and a matrix-core
 * axis that also has an FFT, the candidates are timed with the FFT on such
 * axes as well, and the engines of the fastest are kept
 * (problem_dst_engines reports them).  Blocks until done; out may be NULL
 * (its grid_size is the single-solve grid). */
csl_status problem_tune(csl_problem p, const double *f, double *z,
                        csl_batch_tuning *out, hipStream_t s);

/* Autotuner of the batch schedule: solves the batch for f (results in z)
 * with each candidate tile size, LDS budget and allowed workgroup size,
 * timing every candidate on stream s, and keeps the fastest for later
 * batch_solve calls (the graph is recaptured).  Blocks until done; out may
 * be NULL. */
csl_status batch_tune(csl_batch b, const double *const *f, double *const *z,
                      csl_batch_tuning *out, hipStream_t s);

/* Schedule in use for the problem's own solves / for the batch (host
 * state only; no device work). */
csl_status problem_schedule(csl_problem p, csl_batch_tuning *out);
csl_status batch_schedule(csl_batch b, csl_batch_tuning *out);

csl_status batch_destroy(csl_batch b);

/* ---- The alpha-circulant all-at-once layer (Section 1) ------------------
 * The setting the paper's introduction gives for complex-shifted systems:
 * implicit Euler with step tau for u' + K u = g over L steps, with the
 * bidiagonal time factor (I - Z)/tau replaced by the alpha-circulant
 * C = (I - Z_alpha)/tau (Z_alpha: the down-shift with alpha in its
 * top-right corner).  paradiag_solve applies (kron(C, I) + kron(I, K))^-1:
 *   Rt = (F Gamma (x) I) r,  Gamma = diag(alpha^(k/L)), F the DFT over steps;
 *   (K + D_j I) Ut_j = Rt_j for every mode j, one batched persistent solve,
 *     D_j = (1 - alpha^(1/L) exp(-2 pi i j / L)) / tau;
 *   u = (Gamma^-1 F^-1 (x) I) Ut.
 * All-at-once vectors are DEVICE arrays of L * M complex values, step-major
 * (step k occupies entries [k M, (k + 1) M), each in the grid layout above). */

/* Create the layer: one problem per mode (shift D_j; grid, coefficient and
 * popts as create_problem, which each of them copies) and one batch over
 * them (bopts as batch_create; NULL for the defaults), plus two all-at-once
 * work vectors.  steps = L, a power of two in [8, 1024]; tau > 0;
 * 0 < alpha_c <= 1.  Synchronises s. */
csl_status paradiag_create(const csl_grid *grid, const double *a_nodal, int steps, double tau,
                           double alpha_c, const csl_problem_opts *popts,
                           const csl_batch_opts *bopts, hipStream_t s, csl_paradiag *out);

/* Shift D_j = alpha + i beta of mode j (host). */
csl_status paradiag_shift(csl_paradiag pd, int j, double *alpha, double *beta);

/* The step transform alone: y = (F Gamma (x) I) x (inverse = 0) or
 * y = (Gamma^-1 F^-1 (x) I) x (inverse = 1).  x, y: device, L * M complex,
 * must not alias. */
csl_status paradiag_transform(csl_paradiag pd, const double *x, double *y, int inverse,
                              hipStream_t s);

/* u = (kron(C, I) + kron(I, K))^-1 r.  r, u: device, L * M complex, must
 * not alias.  infos: NULL, or a host array of L solve records (mode j in
 * infos[j]); with infos the call synchronises s and returns CSL_OK only if
 * every mode converged (u is written in any case). */
csl_status paradiag_solve(csl_paradiag pd, const double *r, double *u, csl_solve_info *infos,
                          hipStream_t s);

/* Autotuner of the mode batch (batch_tune) on the modes of the right-hand
 * side r (device, L * M complex).  Blocks until done; out may be NULL. */
csl_status paradiag_tune(csl_paradiag pd, const double *r, csl_batch_tuning *out, hipStream_t s);

/* The batch over the modes, owned by pd (for batch_schedule). */
csl_status paradiag_batch(csl_paradiag pd, csl_batch *out);

csl_status paradiag_destroy(csl_paradiag pd);

/* Thread-local message describing the last non-OK status of this thread. */
const char *csl_last_error(void);

/* Library version (major * 10000 + minor * 100 + patch). */
int csl_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CSL_H */
