/*
 * minres_cg.h -- C ABI of libminrescg.so, a HIP (gfx950) implementation of
 * the two-level nested MINRES-CG scheme of Manguoglu & Mehrmann, "A robust
 * iterative scheme for symmetric indefinite systems" (Section 2, Algorithm
 * "minres_cg"):
 *
 *   outer:  preconditioned MINRES on A x = b, A sparse symmetric indefinite
 *           with k negative eigenvalues (Section 1, eq. "eq1");
 *   first-level preconditioner M_mr = A + 2 Vhat |Lambda_hat| Vhat^T, SPD
 *           (Section 2), applied approximately by
 *   inner:  preconditioned CG on M_mr z = y (eq. "eq2") with a symmetric,
 *           possibly indefinite second-level preconditioner M_cg ~ A
 *           (Jacobi, incomplete LDL^T(0), learned C C^T), optionally in the
 *           Sherman-Morrison-Woodbury form of Section 2.1 (MINRES-CG*).
 *
 * Conventions for every entry point:
 *   - Pointers named "device" point to GPU memory (hipMalloc / torch CUDA
 *     tensors); "host" pointers to CPU memory.  The caller owns every pointer
 *     it passes; the library copies what it needs during *_create and keeps
 *     no reference to caller memory after a call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     All device work of a call is enqueued on it.  Calls that return results
 *     in host memory (stats) synchronize that stream before returning.
 *   - Dense vectors are contiguous; Vhat is n x k column-major (column j at
 *     Vhat + j*n).  CSR matrices use int32 indices, row_ptr[0] = 0,
 *     row_ptr[n] = nnz, column indices sorted and unique within each row,
 *     the full symmetric pattern stored (both triangles).
 *   - Every function returns an mcg_status (0 = success); nothing throws
 *     across the ABI.  A handle is used by one host thread at a time.
 */
#ifndef MINRES_CG_H
#define MINRES_CG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------------ */
/* Status codes.  Positive values describe how a solve ended (the paper's    */
/* failure marks in Section 4: dagger = iteration cap, double dagger =       */
/* stagnation, asterisk = a scalar became too large or too small); negative  */
/* values are errors in the call itself.                                     */
/* ------------------------------------------------------------------------ */
typedef enum {
  MCG_OK = 0,          /* converged: true relative residual <= rtol          */
  MCG_MAXIT = 1,       /* outer or total inner iteration cap reached         */
  MCG_STAGNATION = 2,  /* true residual did not improve over the window      */
  MCG_BREAKDOWN = 3,   /* rho = r^T M_cg^{-1} r vanished, or beta^2 < 0      */
  MCG_NOT_SPD = 4,     /* p^T M_mr p <= 0: Vhat misses a negative eigenvector */
  MCG_EINVAL = -1,     /* invalid argument (shape, pattern, NaN/Inf input)   */
  MCG_EHIP = -2,       /* a HIP runtime call failed                          */
  MCG_ENOMEM = -3      /* device or host allocation failed                   */
} mcg_status;

/* Arithmetic of the inner CG solve.  The outer MINRES (Lanczos vectors,    */
/* Givens rotations, iterate, true residual) is always FP64.                */
typedef enum {
  MCG_PREC_FP64 = 0,   /* inner CG and its preconditioner in FP64            */
  MCG_PREC_MIXED = 1   /* inner CG, M_mr and M_cg in FP32 (FP32 per-thread   */
                       /* accumulation, FP64 cross-block reductions); the    */
                       /* inner right-hand side is scaled to unit norm at    */
                       /* the FP64 -> FP32 boundary and scaled back after    */
} mcg_precision;

/* Second-level (inner CG) preconditioner kinds. */
typedef enum {
  MCG_PC_NONE = 0,     /* M_cg = I                                           */
  MCG_PC_JACOBI = 1,   /* M_cg = diag(A)  (an approximation of A, Section 2) */
  MCG_PC_ILDL0 = 2,    /* M_cg = L D L^T, incomplete LDL^T with zero fill on */
                       /* A's pattern, signed pivots: the symmetric form of  */
                       /* the ILU(0) of A used in Section 4                  */
  MCG_PC_ILDLP = 3,    /* M_cg = P^T L D L^T P, incomplete LDL^T with 1x1 /  */
                       /* 2x2 symmetric pivoting, fill factor and drop       */
                       /* tolerance: the ILDL^T(fill, drop) of Section 4     */
  MCG_PC_CCT = 4,      /* M_cg^{-1} = C C^T, C lower triangular CSR supplied */
                       /* by the caller (the learned factor)                 */
  MCG_PC_SMW = 0x100   /* flag: add -2 Vhat Lambda_hat^{-1} Vhat^T to        */
                       /* M_cg^{-1} (MINRES-CG*, Section 2.1)                */
} mcg_pc_kind;

/* Parameters of MCG_PC_ILDLP (Section 4: ILDL^T(fill, drop); the defaults
 * 3 and 1e-3 are the ones Section 4.3 names).  fill: column j of L keeps at
 * most ceil(fill * m_j) entries, m_j = the off-diagonal entries of A's
 * pivot column in rows not yet pivoted (fill <= 0: no limit).  drop: an
 * entry l of a new column is dropped when |l| < drop * ||column||_2.
 * sweeps: 0 (default) applies the factor exactly (triangular solves,
 * level-scheduled); s in 1..64 replaces each triangular solve by s Jacobi
 * sweeps (u_j = y - L_s u_{j-1}, u_0 = y, L_s = L - I), i.e. applies
 * P^T S^T D^{-1} S P with S = sum_{i<=s} (-L_s)^i: still symmetric, fully
 * parallel, and exact once s reaches the depth of L's dependencies (not in
 * the paper, which applies the factor exactly). */
typedef struct {
  double fill;
  double drop;
  int32_t sweeps;
} mcg_ildlp_params_t;

typedef struct mcg_solver *mcg_handle_t;
typedef struct mcg_pc *mcg_precond_t;

/* Sparse symmetric A in CSR, device pointers. */
typedef struct {
  int32_t n;
  int64_t nnz;
  const int32_t *row_ptr; /* device, n+1 */
  const int32_t *col;     /* device, nnz */
  const double *val;      /* device, nnz */
} mcg_csr_t;

typedef struct {
  int32_t precision;   /* mcg_precision                                      */
  int32_t spmv_lanes;  /* lanes per CSR row in the SpMV kernels: 0 = choose  */
                       /* from the mean row length, else 2, 4, ..., 64; 1 =  */
                       /* CSR-stream (a tile's nonzeros staged through LDS) */
  int32_t autotune;    /* 1: time every lanes-per-row candidate on this      */
                       /* matrix at create and keep the fastest              */
  int32_t stag_window; /* outer iterations without a 0.1% improvement of    */
                       /* the true residual that end a solve with           */
                       /* MCG_STAGNATION (0 = never)                        */
  int32_t keep_best;   /* 1: a solve that does not converge returns the     */
                       /* iterate with the smallest true residual           */
  int32_t block_size;  /* ILDL0: unknowns per node (the FE-like matrices    */
                       /* have 3); level scheduling works on node blocks    */
  int32_t chunk;       /* inner iterations enqueued between two polls of the */
                       /* device-side stop flag (0 = adaptive)              */
  int32_t profile;     /* 1: bracket every launch of the M_mr-apply kernel  */
                       /* inside solves with HIP events on the solve stream */
                       /* (read back with minres_cg_kernel_time); 2: the   */
                       /* product A p (with p^T A p) instead, when A has a */
                       /* sliced copy (else as 1)                          */
  int32_t mmr_form;    /* M_mr apply inside the CG iteration: 0 = default   */
                       /* (split with a block CSR or sliced ELL copy of A, */
                       /* else fused), or the autotuner's choice when      */
                       /* autotune = 1; 1 = fused kernel (one pass over A  */
                       /* and Vhat); 2 = SpMV + streaming rank-k pass      */
  int32_t spmv_format; /* storage of A for the inner products: 0 = choose:  */
                       /* block CSR when block_size > 1 and every nonzero  */
                       /* block is dense, else sliced ELL (slices of 64    */
                       /* rows, 16-bit column offsets when they fit) when  */
                       /* padding adds at most 25 % and spmv_lanes is 0,   */
                       /* else CSR; 1 = CSR only; 2 = sliced ELL with      */
                       /* 32-bit columns, any padding                      */
  int32_t eager;       /* 1: launch the inner iteration's kernels one by one */
                       /* (always so with profile = 1); 0: replay a HIP     */
                       /* graph of 32 iterations, captured on first use for */
                       /* each preconditioner (the same kernels in the same */
                       /* order, so the results are identical)              */
  int32_t xcd_order;   /* slice order of the sliced block products over the */
                       /* 8 XCDs: 0 = automatic (a section order when the   */
                       /* FP32 vector is larger than one XCD's 4 MB L2 and  */
                       /* touches at least 2 % fewer lines of it than the   */
                       /* launch's own order), 1 = the launch's own order,  */
                       /* 2 = as 0 at any vector size                       */
  int32_t reserved[4];
} mcg_options_t;

/* Fill *opt with the defaults: FP64, heuristic lanes, no autotune,
 * stag_window 10, keep_best 1, block_size 1, adaptive chunk, automatic
 * storage format. */
void minres_cg_default_options(mcg_options_t *opt);

typedef struct {
  int32_t status;          /* mcg_status of the solve                        */
  int32_t outer_its;       /* MINRES iterations                              */
  int64_t inner_its_total; /* CG iterations summed over all inner solves     */
  double final_relres;     /* ||b - A x||_2 / ||b||_2 of the returned x, FP64 */
  double bnorm;            /* ||b||_2                                        */
  int32_t hist_cap;        /* capacity of the three host arrays below (may   */
                           /* be 0 / NULL); entries 0..outer_its are filled  */
  int64_t *inner_its;      /* host: CG iterations of inner solve i           */
  double *relres;          /* host: true relative residual after outer its i */
  double *phibar;          /* host: MINRES estimate ||r||_{M^{-1}} after its i */
} mcg_stats_t;

/* ------------------------------------------------------------------------ */
/* Lifecycle                                                                 */
/* ------------------------------------------------------------------------ */

/* Build a solver for A and the deflation data of Section 2: Vhat (device,
 * n x k column-major, orthonormal approximate invariant subspace of the k
 * negative eigenvalues of A) and lam (device, k values, all < 0).  k may be
 * 0 (then M_mr = A, which must be SPD).  Copies A (and an FP32 shadow of A
 * and Vhat when opt->precision is MCG_PREC_MIXED), chooses the SpMV
 * schedule and allocates the whole solve workspace, so that solves allocate
 * nothing.  Validates the CSR structure (EINVAL on unsorted / out-of-range
 * columns, bad row_ptr) and rejects k > 64 or lam >= 0.  opt may be NULL. */
int minres_cg_create(mcg_handle_t *h, const mcg_csr_t *A, int32_t k, const double *Vhat,
                     const double *lam, const mcg_options_t *opt, void *stream);
void minres_cg_free(mcg_handle_t h);

/* Build the second-level preconditioner M_cg for the matrix of h.
 *   MCG_PC_NONE, MCG_PC_JACOBI: params = NULL (Jacobi: EINVAL on a zero or
 *     missing diagonal entry).
 *   MCG_PC_ILDL0: params = NULL or a const double* pivot tolerance; the
 *     factor is computed from A's values in the order A is given (a pivot
 *     with |d_i| < pivtol * max_j |a_ij| is replaced by sign(d_i) times that
 *     floor) and applied by level-scheduled triangular sweeps over node
 *     blocks of opt->block_size unknowns.  EINVAL when a pivot ends up
 *     exactly zero or non-finite (possible only with pivtol = 0) or pivtol
 *     is negative.
 *   MCG_PC_ILDLP: params = NULL (fill 3, drop 1e-3) or a const
 *     mcg_ildlp_params_t*.  The factor P A P^T ~ L D L^T is computed on the
 *     host, column by column in A's order: Bunch-Kaufman choice of a 1x1 or
 *     2x2 pivot (alpha = (1 + sqrt 17) / 8) on the current Schur complement
 *     column, then dropping and the fill limit (largest entries kept, ties
 *     to the smaller original row); a 1x1 pivot below 1e-8 max|a_ij| in
 *     magnitude becomes that floor with its sign.  Applied as gather,
 *     level-scheduled sweeps with L, the blocks of D^{-1}, sweeps with L^T,
 *     scatter (or, with sweeps > 0, gather, s sparse products with L_s,
 *     the blocks of D^{-1}, s with L_s^T, scatter).  No node blocks
 *     (opt->block_size is not used).  EINVAL on a negative or non-finite
 *     fill or drop, sweeps outside 0..64, a singular 2x2 block or a
 *     non-finite factor entry.
 *   MCG_PC_CCT: params = const mcg_csr_t* holding C (device, lower
 *     triangular, n x n); C and C^T are copied.
 * OR-ing MCG_PC_SMW into kind selects the MINRES-CG* form.  The handle
 * stays valid until minres_cg_precond_free and must not outlive h. */
int minres_cg_precond_create(mcg_precond_t *p, mcg_handle_t h, int32_t kind, const void *params,
                             void *stream);
void minres_cg_precond_free(mcg_precond_t p);

/* ------------------------------------------------------------------------ */
/* The solve (Algorithm "minres_cg")                                         */
/* ------------------------------------------------------------------------ */

/* Solve A x = b.  b: device, n x nrhs doubles, column-major (right-hand
 * side j at b + j n).  x: device, n x nrhs doubles; on entry the initial
 * guesses x0, on return the solutions (the best iterate if a solve did not
 * converge and keep_best is set).  The nrhs right-hand sides are solved one
 * after the other on this handle (for many right-hand sides in one launch:
 * the batched solver below, also for a single system).  Outer MINRES stops when
 * ||b - A x||_2 <= rtol_out ||b||_2, recomputed in FP64 every outer
 * iteration; each inner CG solve starts from z0 = 0 and stops when
 * ||r||_2 <= rtol_in ||y||_2.  maxit_out caps MINRES iterations;
 * maxit_inner_total caps CG iterations over the whole solve (each inner solve
 * is also capped at n); with a budget of 0 no inner solve runs and the solve
 * returns MCG_MAXIT with x = x0.  stats (host, may be NULL): nrhs entries,
 * entry j receives the counts and residual histories of right-hand side j.
 * Returns the worst status of the solves (>= 0) or the first error (< 0;
 * EINVAL for nrhs < 1).  Synchronizes `stream`. */
int minres_cg_solve(mcg_handle_t h, mcg_precond_t p, const double *b, double *x, int32_t nrhs,
                    double rtol_out, double rtol_in, int32_t maxit_out, int64_t maxit_inner_total,
                    mcg_stats_t *stats, void *stream);

/* As minres_cg_solve (nrhs = 1), also recording the inner solves: column i
 * of Y (device, n x cap column-major FP64) receives the right-hand side that
 * MINRES hands to inner solve i (r1 for the first, then the Lanczos vector
 * r2 of Algorithm "minres_cg"), and column i of Z the inner CG's result
 * (z ~ M_mr^{-1} y to rtol_in), for the first cap inner solves that ran at
 * least one iteration.  *count (host, may be NULL) receives the number
 * recorded.  These (residual, inner-CG solution) pairs are the training data
 * of a learned second-level preconditioner (include/mcg_learned.h).  Errors
 * and synchronization as minres_cg_solve. */
int minres_cg_solve_record(mcg_handle_t h, mcg_precond_t p, const double *b, double *x,
                           double rtol_out, double rtol_in, int32_t maxit_out,
                           int64_t maxit_inner_total, double *Y, double *Z, int32_t cap,
                           int32_t *count, mcg_stats_t *stats, void *stream);

/* ------------------------------------------------------------------------ */
/* Many systems, several right-hand sides each, one persistent launch        */
/* ------------------------------------------------------------------------ */

typedef struct mcg_batch *mcg_batch_t;

typedef struct {
  int32_t *status;     /* host, nsys*nrhs (system-major): mcg_status per rhs */
  int32_t *outer_its;  /* host, nsys*nrhs */
  int64_t *inner_its;  /* host, nsys*nrhs: CG iterations over all inner solves */
  double *relres;      /* host, nsys*nrhs: final true relative residual      */
} mcg_batch_stats_t;

/* Build a batched solver for nsys independent systems (Algorithm
 * "minres_cg" applied to each; the paper's setting of many shifted systems,
 * Section 3.1) with nrhs (1..8) right-hand sides each.  As, ks, Vhats, lams
 * are host arrays of nsys entries describing each system as in
 * minres_cg_create (device pointers inside; copied).  Inner preconditioner:
 * Jacobi.  opt->precision selects FP32 or FP64 inner CG (outer always FP64);
 * opt->stag_window and opt->keep_best apply per right-hand side.  Systems
 * are grouped by k (buckets of at most 8, 16, 32, 40, 48, 64 columns); each
 * group is one persistent kernel launch whose grid never exceeds what the
 * GPU keeps resident, and each system gets a team of its group's
 * workgroups in proportion to its work, nnz + (k + 1) n.  EINVAL if a k
 * exceeds 64 or nrhs is outside 1..8. */
int minres_cg_batch_create(mcg_batch_t *b, int32_t nsys, const mcg_csr_t *As, const int32_t *ks,
                           const double *const *Vhats, const double *const *lams, int32_t nrhs,
                           const mcg_options_t *opt, void *stream);
/* The same constructor under the name minres_cg_create_batch. */
int minres_cg_create_batch(mcg_batch_t *b, int32_t nsys, const mcg_csr_t *As, const int32_t *ks,
                           const double *const *Vhats, const double *const *lams, int32_t nrhs,
                           const mcg_options_t *opt, void *stream);

/* Solve every system for its nrhs right-hand sides.  Bs[i], Xs[i]: device,
 * n_i x nrhs column-major (right-hand side j at Bs[i] + j*n_i); Xs[i] holds
 * the initial guesses on entry and the solutions on return.  Stopping rules
 * per right-hand side as in minres_cg_solve; maxit_inner caps each inner
 * solve (also capped at n_i; 0: no inner solve runs, every right-hand side
 * ends with MCG_MAXIT and x = x0).  use_graph = 1 captures the whole sequence
 * (layout conversions, counter resets via kernels, the persistent kernel)
 * into a hipGraph on the first call for a given set of Bs/Xs pointers and replays
 * it afterwards (the tolerances and caps must then stay the same, else
 * EINVAL).  Returns the worst per-rhs status (>= 0) or an error; a team that
 * waited on a barrier for more than 20 s aborts the launch (MCG_EHIP) instead
 * of hanging.  Synchronizes `stream`. */
int minres_cg_batch_solve(mcg_batch_t b, const double *const *Bs, double *const *Xs,
                          double rtol_out, double rtol_in, int32_t maxit_out, int64_t maxit_inner,
                          int32_t use_graph, mcg_batch_stats_t *stats, void *stream);

/* The same batched solve run as independent single-system solves (the
 * kernels of minres_cg_solve) on nstreams HIP streams (1..16), one host
 * worker thread per stream; systems are assigned longest first by their
 * estimated work (nnz + (k + 1) n per right-hand side) and each stream solves
 * its systems' right-hand sides in turn.  Many small systems then overlap on
 * the GPU without the device-wide barriers of the persistent launch.  Bs, Xs,
 * st and the return value as for minres_cg_batch_solve, except that
 * maxit_inner caps the CG iterations of each right-hand side's whole solve
 * (as maxit_inner_total of minres_cg_solve).  The handles' Jacobi
 * preconditioners serve as M_cg.  The calling thread
 * waits for all streams; work already queued on `stream` is waited for
 * first. */
int minres_cg_batch_solve_streams(mcg_batch_t B, const double *const *Bs, double *const *Xs,
                                  double rtol_out, double rtol_in, int32_t maxit_out,
                                  int64_t maxit_inner, int32_t nstreams, mcg_batch_stats_t *st,
                                  void *stream);

/* The single-system handle of system i of the batch (owned by the batch,
 * valid until minres_cg_batch_free), on which second-level preconditioners
 * of any kind (ILDL0, ILDLP, CCT, SMW) can be created for the stream mode
 * below.  EINVAL for i outside 0..nsys-1. */
int minres_cg_batch_system(mcg_batch_t b, int32_t i, mcg_handle_t *h);

/* minres_cg_batch_solve_streams with a second level per system: pcs (host,
 * nsys entries) holds preconditioners created on minres_cg_batch_system(b,
 * i), or NULL for the batch's Jacobi.  Each system's preconditioner is used
 * by one worker thread at a time; a preconditioner must not be shared
 * between systems (EINVAL when pcs[i] belongs to another handle). */
int minres_cg_batch_solve_streams_pc(mcg_batch_t b, const mcg_precond_t *pcs,
                                     const double *const *Bs, double *const *Xs, double rtol_out,
                                     double rtol_in, int32_t maxit_out, int64_t maxit_inner,
                                     int32_t nstreams, mcg_batch_stats_t *st, void *stream);

/* Re-plan the teams of the persistent launches: system i's share of its
 * group's workgroups becomes proportional to weights[i] * (nnz + (k + 1) n)
 * (weights: host, nsys values > 0).  Meant for repeated solves of the same
 * systems, with weights[i] the inner CG iterations system i took in an
 * earlier solve (its team's count from minres_cg_batch_profile, or the
 * largest over its right-hand sides), so that teams finish together rather
 * than in proportion to their matrix sizes. Results
 * stay correct for any weights; reduction order follows the teams, so they
 * may change in the last bits.  Drops a captured graph (the next use_graph
 * solve captures again).  Call between solves only (copies synchronously).
 * EINVAL for a non-positive or non-finite weight. */
int minres_cg_batch_rebalance(mcg_batch_t b, const double *weights);

/* Re-plan the persistent launches' teams from the block-time each system
 * took in the last persistent solve (its team's wall-clock span times its
 * team size, from the clocks minres_cg_batch_profile reports): each launch's
 * blocks are handed out one at a time to the team whose predicted span
 * (block-time / team size) is the longest, which minimises the launch's
 * longest predicted span over integer team sizes.  Unlike iteration counts,
 * block-times also carry what a team's speed owes to its size.  Call between
 * solves only (copies synchronously); a team that ended within one clock
 * tick counts one tick.  EINVAL when no persistent solve ran since the batch
 * was created. */
int minres_cg_batch_rebalance_measured(mcg_batch_t b);

/* Timing of the last persistent solve (minres_cg_batch_solve), per system
 * (host arrays of nsys, each may be NULL): the GPU wall clock when its team
 * started and ended, the inner CG iterations the team ran (counted once per
 * iteration, whatever the number of right-hand sides still active), the
 * wall-clock ticks the team's first workgroup spent in the inner
 * iteration's three phases (phase_ticks: 6 per system -- SpMM with the
 * rank-k part, then its team reduction; the z / r update, then its
 * reduction; the direction update, then its barrier or refresh reduction),
 * and the index of the system's launch (k bucket, launches in order).
 * clock_hz (may be NULL) receives the wall clock's rate.  Zeros before the
 * first persistent solve.  Call after the solve returned (copies
 * synchronously). */
int minres_cg_batch_profile(mcg_batch_t b, int64_t *t_begin, int64_t *t_end, int64_t *team_iters,
                            int64_t *phase_ticks, int32_t *group, double *clock_hz);

/* Launch shape: total workgroups and the team size of each system (host
 * array of nsys, may be NULL). */
int minres_cg_batch_info(mcg_batch_t b, int32_t *nblocks, int32_t *team_sizes);

void minres_cg_batch_free(mcg_batch_t b);

/* ------------------------------------------------------------------------ */
/* Steps of the hot path, exposed one by one                                 */
/* ------------------------------------------------------------------------ */

/* y = A x.  precision MCG_PREC_FP64: x, y are device double[n] and A's FP64
 * values are used; MCG_PREC_MIXED: x, y are device float[n] and the FP32
 * shadow of A is used (EINVAL if h was not created with MCG_PREC_MIXED). */
int mcg_spmv(mcg_handle_t h, int32_t precision, const void *x, void *y, void *stream);

/* q = M_mr u = A u + 2 Vhat (|Lambda_hat| (Vhat^T u)) (Section 2, the
 * product used by every CG iteration).  Vectors as in mcg_spmv. */
int mcg_mmr_apply(mcg_handle_t h, int32_t precision, const void *u, void *q, void *stream);

/* t = M_cg^{-1} g for the preconditioner p (precision as in mcg_spmv).  g and
 * t are either the same array (in place) or do not overlap. */
int mcg_precond_apply(mcg_precond_t p, int32_t precision, const void *g, void *t, void *stream);

/* The MCG_PC_ILDLP factor of p, copied to host arrays (P A P^T ~ L D L^T,
 * Section 4): perm[k] = original index of logical row k; bsize[k] = 1 (1x1
 * pivot), 2 (first row of a 2x2 pivot) or 0 (its second row); dd = D's
 * diagonal, doff[k] = D(k, k+1) at the first row of a 2x2 block (0
 * elsewhere); L strictly lower in logical CSR (l_ptr n+1, l_col / l_val
 * nnz_l, columns ascending).  Arrays may be NULL to query *nnz_l (host,
 * required) first; l_col / l_val must hold *nnz_l entries on entry when
 * given.  EINVAL when p is not an MCG_PC_ILDLP preconditioner. */
int mcg_ildlp_factor_get(mcg_precond_t p, int32_t *perm, int32_t *bsize, double *dd, double *doff,
                         int32_t *l_ptr, int32_t *l_col, double *l_val, int64_t *nnz_l);

/* One inner solve: z = PCG(M_mr, M_cg = p; y), z0 = 0, stop at
 * ||r|| <= rtol_in ||y|| or maxit iterations.  y, z: device double[n]; in
 * MCG_PREC_MIXED the solve runs in FP32 behind the scaling boundary.
 * *its (host, may be NULL) receives the iteration count.  Returns MCG_OK,
 * MCG_MAXIT, MCG_BREAKDOWN or MCG_NOT_SPD; maxit = 0 gives z = 0 and
 * MCG_MAXIT (y = 0: z = 0 and MCG_OK).  Synchronizes `stream`. */
int mcg_pcg_solve(mcg_handle_t h, mcg_precond_t p, const double *y, double *z, double rtol_in,
                  int64_t maxit, int64_t *its, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the M_mr
 * apply of mcg_mmr_apply in FP64, q = A u + 2 Vhat (|lam| o (Vhat^T u)),
 * taken straight from the caller's arrays, with no handle and no allocation.
 * A: device CSR as in minres_cg_create; Vhat: device, n x k column-major;
 * lam: device, k values (used as |lam_j|); u, q: device double[n] (q must not
 * overlap u).  k = 0 gives q = A u.  EINVAL for k outside 0..64, n k >= 2^31
 * or missing pointers (nothing is validated on the device: no value of A,
 * Vhat or lam is read back, so the call can be captured in a graph once the
 * library has been used on the device).  Its only workspace is a fixed
 * device array of the library (1024 x 64 + 64 doubles per GPU, held until
 * the process ends) that every call overwrites; calls that overlap on one
 * GPU race on it.  Asynchronous on `stream`. */
int mcg_mmr_apply_noalloc(const mcg_csr_t *A, int32_t k, const double *Vhat, const double *lam,
                          const double *u, double *q, void *stream);

/* Accumulated device time of the M_mr-apply kernel (the fused SpMV +
 * low-rank product that dominates each CG iteration) over the solves run
 * since the last reset, counting only launches that did work (launches
 * enqueued after the inner solve had stopped are excluded).  Requires
 * opt->profile != 0 at create; *ms and *launches are host pointers.
 * reset = 1 clears the counters after reading. */
int minres_cg_kernel_time(mcg_handle_t h, double *ms, int64_t *launches, int32_t reset);

/* Lanes per CSR row the SpMV kernels of h use (chosen at create by the
 * mean-row-length rule, opt->spmv_lanes, or the autotuner). */
int minres_cg_spmv_lanes(mcg_handle_t h);

/* 1 if the M_mr apply of the Jacobi-preconditioned iteration runs as an SpMV
 * followed by a streaming rank-k pass (chosen by the autotuner when faster on
 * this matrix), 0 if fused in one kernel, -1 for a NULL handle. */
int minres_cg_mmr_split(mcg_handle_t h);

/* Block size of the block CSR copy of A that the inner SpMVs use (opt
 * block_size 2..4 when every nonzero block of A is dense), or 0 when A is
 * used in CSR form only. */
int minres_cg_block_csr(mcg_handle_t h);

/* Column index width in bits (16 or 32) of the sliced ELL copy of A that the
 * inner SpMVs and M_mr applies use, 0 when there is none, -1 for a NULL
 * handle. */
int minres_cg_sliced_ell(mcg_handle_t h);

/* Block size of the sliced block copy of A (built next to the block CSR
 * copy when slice padding adds at most 25 %), 0 when there is none, -1 for
 * a NULL handle. */
int minres_cg_sliced_blocks(mcg_handle_t h);

/* Slice order of the sliced block SpMV over the 8 XCDs (each with its own
 * L2): P > 0 when XCD e takes the e-th eighth of each of P equal sections of
 * the slices (chosen at create time as the candidate whose XCDs touch the
 * fewest 128-byte lines of x; see mcg_options_t.xcd_order), 0 when the
 * launch's own round-robin order is kept, -1 for a NULL handle or no sliced
 * block copy. */
int minres_cg_xcd_sections(mcg_handle_t h);

/* ------------------------------------------------------------------------ */
/* Host-only queries (no GPU needed)                                         */
/* ------------------------------------------------------------------------ */

/* Number of length-n vectors the solve keeps in device memory, excluding A,
 * the preconditioner and b, counted the way the paper's storage table
 * counts them (MINRES 7, MINRES-CG 11 + k): *paper receives 11 + k, *total
 * the vectors this implementation actually allocates (it adds the true
 * residual, the best iterate and, in mixed precision, FP32 copies). */
int minres_cg_workspace_vectors(int32_t k, int32_t precision, int32_t pc_kind, int32_t *paper,
                                int32_t *total);

/* Static text for a status code. */
const char *minres_cg_strerror(int code);

/* Library version, e.g. "minres_cg 1.0 gfx950". */
const char *minres_cg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MINRES_CG_H */
