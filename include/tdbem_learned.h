/*
 * tdbem_learned.h -- learned variable preconditioner for the FGMRES solve of tdbem.h.
 *
 * Not part of the paper.  Flexible GMRES (Saad 1993), which the paper uses in Section 4.2 so
 * that its block-Hessenberg preconditioner (Algorithm 1) may change between iterations, accepts
 * any nonlinear map z = P(v) as a right preconditioner.  This one is a message-passing network on
 * the space-time graph of the unknowns: node (k, j) is the coefficient of b_k phi_j, index k*M+j
 * in the vectors of tdbem.h.  A node exchanges messages with its mesh neighbours (vertices that
 * share an edge) in time block k and with (k-1, j), (k+1, j).
 *
 *   s = sqrt(mean(v^2));  x(k,j) = [v(k,j)/s, h_k/hbar, h_{k+1}/hbar]   (h_k = t_k - t_{k-1},
 *                                                                        0 outside; hbar = T/(N-1))
 *   H = Win x + bin;  for each layer: U = W [H, mean_nbrs H, H(k-1), H(k+1)] + b;  H += relu(U)
 *   z = s * (wout . H)
 *
 * 64 channels per node, float32 activations and accumulation, bfloat16 weights (Win, W, wout
 * rounded to nearest even from float32 master copies), float32 biases.  Flat parameter layout
 * (float32): Win[64][3], bin[64], then per layer W[64][256] (feature blocks in the order above)
 * and b[64], then wout[64]: 256 + layers*16448 + 64 values.
 *
 * Training (tdbem_lp_train) minimises the mean over a batch of ||A P(v) - v||^2 / ||v||^2 with
 * Adam on the GPU; the residuals v are drawn by the library: standard normal vectors and
 * products A x of normal vectors x smoothed over the mesh.  The gradient needs A^T, provided by
 * tdbem_matvec_transpose.  Weights do not depend on the mesh or the grid: a network trained on
 * one problem can be applied to another.
 */
#ifndef TDBEM_LEARNED_H
#define TDBEM_LEARNED_H

#include <stdint.h>

#include "tdbem.h"

#ifdef __cplusplus
extern "C" {
#endif

#define TDBEM_LP_MAX_LAYERS 8

typedef struct {
    int32_t steps;               /* Adam steps */
    int32_t batch;               /* residuals per step */
    double lr;                   /* Adam learning rate (e.g. 1e-3) */
    uint64_t seed;               /* seed of the residual generator */
} tdbem_lp_train_opts;

typedef struct {
    int32_t steps;
    int64_t samples;             /* residuals used */
    double loss_first, loss_last;/* mean loss of the first and of the last step */
    double ms;                   /* wall time */
} tdbem_lp_train_report;

/* Number of parameters of a network with `layers` message-passing layers (1..8), -1 otherwise. */
int64_t tdbem_lp_num_params(int32_t layers);

/* (Re)initialise the network of ctx: `layers` layers (1..8), uniform random weights from `seed`
 * (+-1/sqrt(3) for Win and bin, +-0.3/16 for the layer weights and biases, +-1/8 for wout); resets
 * the Adam state.  TDBEM_EINVAL for a bad layer count. */
tdbem_status tdbem_lp_init(tdbem_ctx *ctx, int32_t layers, uint64_t seed);

/* Copy n = tdbem_lp_num_params(layers) float32 parameters from / to the host (layout above).
 * set_params resets the Adam state.  TDBEM_ESTATE before tdbem_lp_init, TDBEM_EINVAL for a
 * wrong n. */
tdbem_status tdbem_lp_set_params(tdbem_ctx *ctx, const float *params, int64_t n);
tdbem_status tdbem_lp_get_params(tdbem_ctx *ctx, float *params, int64_t n);

/* z = P(v) for device vectors of N*M float64 on the current mesh and grid (no assembly needed;
 * v = 0 gives z = 0). */
tdbem_status tdbem_lp_apply(tdbem_ctx *ctx, const double *v, double *z);

/* z = P(v) and the gradient of <dz, P(v)> with respect to the parameters: v, dz, z device vectors
 * of N*M float64, grad a host array of tdbem_lp_num_params(layers) floats (overwritten).  The
 * bfloat16 rounding is taken as the identity (the gradient at the rounded weights). */
tdbem_status tdbem_lp_gradient(tdbem_ctx *ctx, const double *v, const double *dz, double *z, float *grad);

/* x = A^T y for device vectors of N*M float64 (every block A_{k,i} is symmetric, so
 * (A^T y)_i = sum_k A_{k,i} y_k).  Requires tdbem_assemble. */
tdbem_status tdbem_matvec_transpose(tdbem_ctx *ctx, const double *y, double *x);

/* Train the network on the assembled operator of ctx (see above).  loss_history (host, may be
 * NULL) receives opts->steps mean losses; rep may be NULL.  TDBEM_ESTATE before tdbem_lp_init or
 * tdbem_assemble. */
tdbem_status tdbem_lp_train(tdbem_ctx *ctx, const tdbem_lp_train_opts *opts, float *loss_history,
                            tdbem_lp_train_report *rep);

#ifdef __cplusplus
}
#endif

#endif /* TDBEM_LEARNED_H */
