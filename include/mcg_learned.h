/* Learned second-level preconditioner for the inner CG of MINRES-CG.
 *
 * The paper's inner solve (Section 2, the CG on M_mr = A + 2 Vhat |Lambda_hat|
 * Vhat^T, Algorithm "minres_cg") may itself be preconditioned by any SPD
 * M_cg.  This library adds one that is learned: a message-passing network
 * over the node graph of A outputs a lower-triangular C on the pattern of
 * lower(A) with a positive diagonal, and M_cg^{-1} = C C^T, which is SPD by
 * construction for any network weights.  The paper itself contains no
 * learned component; the network below is this library's own definition.
 *
 * Network (H = 32 hidden features, bs unknowns per node, nodes I, J):
 *   s_i = sqrt|a_ii|, At = S^-1 A S^-1
 *   x_I  = lower triangle of At's diagonal block (row-major, bs(bs+1)/2)
 *   f_IJ = the bs x bs block At_IJ, I != J (row-major)
 *   h_I = W_in_n x_I,  e_IJ = W_in_e f_IJ
 *   4 layers: m_IJ = relu(W1 [h_I; h_J; e_IJ] + b1);  e_IJ += m_IJ;
 *             a_I = sum_J m_IJ;  h_I += relu(W2 [h_I; a_I] + b2)
 *   C block (I, J), J < I:  0.1 * reshape(W_oe e_IJ)
 *   C diagonal block I:     o = W_od h_I + b_od; diagonal softplus(o) + 1e-3,
 *                           strictly lower 0.1 * o
 *   C = S^-1 Ct (row scaling)
 * Training loss for pairs (y_b, z_b), b < nb:
 *   L = (1/nb) sum_b ||C C^T y_b - z_b||^2 / ||z_b||^2.
 *
 * Parameters: one FP32 vector (master copy), in the order
 *   W_in_n (H x dn), W_in_e (H x de), then per layer W1 (H x 3H), b1 (H),
 *   W2 (H x 2H), b2 (H), then W_oe (de x H), W_od (dn x H), b_od (dn),
 * all row-major, dn = bs(bs+1)/2, de = bs*bs.  The network computes with the
 * weights rounded to bfloat16 (round to nearest even); hidden layers run on
 * BF16 matrix cores with FP32 accumulation, activations are kept in FP32.
 * Gradients are those of the loss with respect to the rounded weights.
 *
 * All pointers are device pointers unless marked host.  Calls are
 * asynchronous on `stream` (a hipStream_t, NULL = default) except where a
 * host result is returned.  Errors: MCG_EINVAL for bad shapes or patterns,
 * MCG_ENOMEM, MCG_EHIP (see mcg_status in minres_cg.h).
 */
#ifndef MCG_LEARNED_H
#define MCG_LEARNED_H

#include "minres_cg.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mcg_learned *mcg_learned_t;

/* Builds the node graph of A (CSR, device, symmetric pattern with a nonzero
 * diagonal, n a multiple of block_size, 1 <= block_size <= 4, at most 64
 * neighbour nodes per node) and allocates every buffer of the network.  The
 * graph build runs on the host (A's arrays are copied down once).  The
 * parameters start at zero; set them with mcg_learned_set_params.  The
 * handle does not reference A after the call returns. */
int mcg_learned_create(mcg_learned_t *out, const mcg_csr_t *A, int32_t block_size, void *stream);
void mcg_learned_free(mcg_learned_t h);

/* Number of FP32 parameters (see the layout above). */
int64_t mcg_learned_num_params(mcg_learned_t h);
/* Graph sizes: nodes, directed edges (I != J), nonzeros of C (host outputs,
 * any may be NULL). */
int mcg_learned_sizes(mcg_learned_t h, int64_t *nodes, int64_t *edges, int64_t *nnz_c);

/* Copies P FP32 parameters in / out (device arrays of num_params floats). */
int mcg_learned_set_params(mcg_learned_t h, const float *theta, void *stream);
int mcg_learned_get_params(mcg_learned_t h, float *theta, void *stream);

/* Network inference: computes C.  Afterwards mcg_learned_factor exposes C. */
int mcg_learned_forward(mcg_learned_t h, void *stream);

/* C of the last forward as a CSR (device pointers owned by the handle, valid
 * until the next forward or free): lower triangular, rows in A's order,
 * entries in A's order within each row, FP64 values.  This is the params
 * argument of minres_cg_precond_create(..., MCG_PC_CCT, ...). */
int mcg_learned_factor(mcg_learned_t h, mcg_csr_t *C);

/* Copies C of the last forward into caller-owned device arrays of n+1,
 * nnz_c and nnz_c elements. */
int mcg_learned_factor_copy(mcg_learned_t h, int32_t *row_ptr, int32_t *col, double *val,
                            void *stream);

/* Forward, loss and backward for nb pairs (1 <= nb <= 32, a power of two):
 * Y and Z are n x nb FP32, row-interleaved (element (i, b) at i*nb + b).
 * *loss (host) receives L (the call waits for the stream); grad (may be NULL)
 * receives dL/dtheta (num_params floats). */
int mcg_learned_loss_grad(mcg_learned_t h, const float *Y, const float *Z, int32_t nb,
                          double *loss, float *grad, void *stream);

/* One Adam step on caller-held FP32 arrays of P elements: theta -= lr *
 * mhat / (sqrt(vhat) + eps) with m1, m2 the first and second moments
 * (updated in place) and bias correction for step (counted from 1).  Used
 * with the gradient of mcg_learned_loss_grad; training over several
 * matrices shares one theta / m1 / m2 between their handles. */
int mcg_learned_adam(int64_t P, float *theta, const float *grad, float *m1, float *m2, float lr,
                     float beta1, float beta2, float eps, int32_t step, void *stream);

/* Device time (ms, HIP events) of the last forward's message-passing
 * kernels, or -1 when no forward has been timed. */
double mcg_learned_forward_ms(mcg_learned_t h);

#ifdef __cplusplus
}
#endif
#endif
