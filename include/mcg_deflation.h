/* Setup stage of MINRES-CG on the GPU: the deflation data (V-hat, Lambda-hat).
 *
 * The method needs an approximate invariant subspace of A for its k negative
 * eigenvalues (Section 2: M_mr = A + 2 V-hat |Lambda-hat| V-hat^T is SPD when
 * V-hat spans the negative eigenvectors); the paper computes it once per
 * matrix with a sparse eigensolver (Section 4) and amortises it over many
 * solves (Section 3.2).  This entry point computes the k algebraically
 * smallest eigenpairs of a sparse symmetric A on the device, by
 * Chebyshev-filtered subspace iteration with Rayleigh-Ritz (Zhou, Saad,
 * Tiago and Chelikowsky, 2006): a block of p >= k vectors is filtered by a
 * polynomial that damps A's spectrum above the block's largest Ritz value,
 * orthonormalised (Cholesky QR, twice) and rotated onto its Ritz vectors,
 * until the k wanted eigen-residuals reach the tolerance.
 *
 * All pointers to A are device pointers (mcg_csr_t of minres_cg.h); the
 * library copies what it needs and keeps nothing after return.
 */
#ifndef MCG_DEFLATION_H
#define MCG_DEFLATION_H

#include <stdint.h>

#include "minres_cg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t block;     /* subspace size p: 0 = k + max(8, k/2); rounded up to */
                     /* a multiple of 16; at most 64                        */
  int32_t degree;    /* Chebyshev polynomial degree per outer iteration     */
                     /* (0 = 64)                                            */
  int32_t max_outer; /* outer iterations (filter + Rayleigh-Ritz), 0 = 400  */
  int32_t reserved0;
  double tol;        /* target: every wanted eigen-residual                 */
                     /* ||A v - theta v|| <= tol * g, g = the Gershgorin     */
                     /* bound max_i sum_j |a_ij| (0 = 1e-10)                */
  uint64_t seed;     /* start block: counter-based uniform numbers          */
} mcg_eig_options_t;

typedef struct {
  int32_t outer_its;   /* outer iterations done                             */
  int32_t spmm_calls;  /* block products A X                                */
  int32_t negative;    /* Ritz values among the k returned that are < 0     */
  int32_t converged;   /* 1 if the tolerance was reached                    */
  double max_residual; /* max_j ||A v_j - theta_j v_j|| over the k returned */
  double bound;        /* the Gershgorin bound g                            */
  double next_ritz;    /* Ritz value k + 1 (the first one not returned)     */
} mcg_eig_stats_t;

/* Fill *opt with the defaults (all zero: the defaults listed above). */
void minres_cg_eig_default_options(mcg_eig_options_t *opt);

/* The k smallest eigenpairs of A (k >= 1, k + 8 <= 64 with the default
 * block).  Vhat: device, n x k, column-major (the layout minres_cg_create
 * takes), orthonormal columns in ascending order of the eigenvalues; lam:
 * host, k values ascending.  A must be symmetric (only its CSR pattern and
 * values are read; symmetry is not checked) with sorted columns.  Returns
 * MCG_OK (stats->converged tells whether the tolerance was reached within
 * max_outer), MCG_BREAKDOWN if the filtered block lost rank (Cholesky QR
 * failed even with a diagonal shift), MCG_EINVAL for bad arguments (k < 1,
 * p > 64, p > n, invalid CSR, non-finite values), MCG_ENOMEM / MCG_EHIP on
 * device errors.  Device workspace: about
 * 5 n p doubles, freed before return.  Synchronizes `stream`. */
int minres_cg_lowest_eigs(const mcg_csr_t *A, int32_t k, const mcg_eig_options_t *opt,
                          double *Vhat, double *lam, mcg_eig_stats_t *stats, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MCG_DEFLATION_H */
