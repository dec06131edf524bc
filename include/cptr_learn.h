/*
 * cptr_learn.h -- learned second stage of libcptr (not in the paper).
 *
 * A small message-passing network on the 7-point cell graph replaces the
 * ILU(0) second stage M2^{-1} of the two-stage preconditioner (Section 3,
 * "Two-stage preconditioners": z = M2^{-1} b1 + x1).  Hidden width 64, three
 * layers, BF16 matrix-core products with FP32 accumulation:
 *   r = D^{-1} b1 (D: diagonal blocks of A), s_k = RMS over cells of r_k for
 *   each unknown k (they have different units), u_k = r_k / s_k
 *   e_{i,d} = S^{-1} D_i^{-1} A_{i,nbr(i,d)} S, S = diag(s_k) (the block in
 *             the scaled unknowns), d = (-x,+x,-y,+y,-z,+z) ordered by the
 *             column offset of the neighbour (zero when absent)
 *   h0 = W_in u;  for l = 1..3:  m_i = sum_d (W_e e_{i,d}) * h_{nbr(i,d)},
 *                 h_i <- h_i + relu(W_s h_i + W_m m_i + b)
 *   z2_k = s_k (u_k + (W_out h3)_k)
 * Parameters: one FP32 vector, layout W_in (64 x nv), then for each layer
 * W_e (64 x nv^2), W_s (64 x 64), W_m (64 x 64), b (64), then W_out (nv x 64),
 * all row-major.  W_out = 0 makes the stage block Jacobi.
 * Training minimises the mean over pairs of ||b1 - A z2||^2 / ||b1||^2 with
 * Adam; every step runs on the device (forward, A^T product, backward,
 * deterministic gradient reductions, Adam).
 * A handle set up with CPTR_SECOND_LEARNED applies the attached model and
 * falls back to BILU(0) in natural order (plain ILU(0)-CPTR) if the stage
 * produces a non-finite value or if a whole FGMRES cycle fails to halve the
 * true residual (cptr_solve_info.fell_back).  Pointers are device pointers unless named
 * *_host; status codes as in cptr.h.
 */
#ifndef CPTR_LEARN_H
#define CPTR_LEARN_H

#include <stddef.h>

#include "cptr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cptr_learn_model cptr_learn_model;

/* Number of FP32 parameters for nv unknowns per cell (nv = 3 or 4). */
size_t cptr_learn_param_count(int nv);

/* New model on the current device with parameters theta_host (host FP32,
 * cptr_learn_param_count(nv) values).  Adam state starts at zero. */
int cptr_learn_create(cptr_learn_model **out, int nv, const float *theta_host);
/* Replace the parameters (host, count as above).  New parameters start a new
 * optimisation: the Adam moments and step count are reset to zero. */
int cptr_learn_set_params(cptr_learn_model *m, const float *theta_host);
int cptr_learn_get_params(const cptr_learn_model *m, float *theta_host);
void cptr_learn_destroy(cptr_learn_model *m);

/* Use m for the learned stage of h (and for the calls below).  The model
 * must outlive its use by h; nv must match.  Builds the matrix data of the
 * stage on first use (neighbour table, edge features).  A handle of any
 * second stage may be attached for training; only CPTR_SECOND_LEARNED
 * handles apply the model inside cptr_apply / fgmres_solve.  Attaching (again)
 * also re-enables the learned stage of a handle that fell back to BILU(0). */
int cptr_learn_attach(cptr_handle *h, cptr_learn_model *m);

/* z2 = N(b1) for one vector (device FP64 [n*nv] in and out).  Asynchronous. */
int cptr_learn_forward(cptr_handle *h, const double *b1, double *z2, void *stream);

/* Launch layer `layer` (0, 1 or 2) of the most recent inference pass of h
 * (cptr_learn_forward, or the learned stage inside cptr_apply / fgmres_solve)
 * once more on `stream`.  Its inputs are unchanged, so it rewrites the same
 * values; layer 2 writes z2 = N(b1) of that pass to `z2` (device FP64
 * [n*nv]; may be NULL for layers 0 and 1).  A measurement aid: it times one
 * layer kernel alone.  CPTR_ERR_INVALID_ARG before any inference pass or for
 * a layer out of range.  Asynchronous. */
int cptr_learn_rerun_layer(cptr_handle *h, int layer, double *z2, void *stream);

/* Mean loss over `count` vectors b1 (device FP64, count x n*nv, back to back)
 * and its gradient (grad_host: host FP32, cptr_learn_param_count values, or
 * NULL).  Blocking. */
int cptr_learn_grad(cptr_handle *h, const double *b1, int count, float *loss_host,
                    float *grad_host, void *stream);

/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on the mean gradient
 * over `count` vectors b1; loss_host receives the mean loss before the step.
 * Blocking. */
int cptr_learn_train_step(cptr_handle *h, const double *b1, int count, float lr, float *loss_host,
                          void *stream);

#ifdef __cplusplus
}
#endif
#endif
