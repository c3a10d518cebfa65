/* Pricing surrogate on MI355X: a 6-256-256-256-1 perceptron trained on
 * quantization-tree prices (C ABI).
 *
 * The tree of qtree.h prices one contract per solve: transition weights
 * (Sec. 3 / 4) and the backward dynamic programming (Sec. 2).  The surrogate
 * maps the contract parameters x = (S0/K, sigma, r, T, n, rho) to the tree
 * price V_0 / K, so that a query inside the training box [lo, hi] costs one
 * network evaluation; a query outside it is flagged so that the caller can
 * price it with the tree.
 *
 * Network (parameters packed in one FP32 vector, rows = output units):
 *   u   = 2 (x - lo) / (hi - lo) - 1        (0 in a slot with hi = lo)
 *   z1  = W1 u + b1,      h1 = silu(z1)     W1: [256][6]      (VALU)
 *   z2  = W2 h1 + b2,     h2 = silu(z2)     W2: [256][256]    (bf16 MFMA)
 *   z3  = W3 h2 + b3,     h3 = silu(z3)     W3: [256][256]    (bf16 MFMA)
 *   y   = s (w4 . h3 + b4) + base(x)        w4: [256], b4     (VALU)
 * silu(z) = z / (1 + e^-z).  base is 0, or (baseline = 1) the Black-Scholes
 * value of the European put per unit strike on the raw inputs
 * x = (S0/K, sigma, r, T, ...):  e^{-rT} Phi(-d2) - (S0/K) Phi(-d1),
 * d1 = (ln(S0/K) + (r + sigma^2/2) T) / (sigma sqrt(T)), d2 = d1 - sigma sqrt(T)
 * (FP32; a control variate: the network then learns the early-exercise
 * premium and the tree's own bias).  Offsets in the packed vector: W1 0, b1 1536,
 * W2 1792, b2 67328, W3 67584, b3 133120, w4 133376, b4 133632; 133633 in
 * all.  The weight matrices are used as BF16 (the FP32 master copy rounded
 * to nearest even after every update); biases are FP32; accumulation is
 * FP32.  The activations entering the two MFMA layers are split into
 * `act_terms` BF16 numbers (1: h rounded once; 2: hi = bf16(h) and
 * lo = bf16(h - hi), ~16 significant bits, twice the MFMA work).
 *
 * Ownership: the caller owns every device buffer (inputs, outputs and the
 * workspace, which holds the parameters, Adam moments, BF16 copies and the
 * training activations).  All validation happens on the host before any
 * device work; errors leave outputs untouched.  Calls are asynchronous on
 * `stream` (a hipStream_t; NULL = the default stream) unless stated.
 * Calls that share one qtree_mlp must not overlap (they share its buffers).
 * ---------------------------------------------------------------------- */
#ifndef QTREE_MLP_H
#define QTREE_MLP_H

#include <stddef.h>
#include <stdint.h>

#include "qtree.h"

#ifdef __cplusplus
extern "C" {
#endif

#define QTREE_MLP_INPUTS 6
#define QTREE_MLP_HIDDEN 256
#define QTREE_MLP_PARAMS 133633

typedef struct qtree_mlp qtree_mlp;

/* Adam hyper-parameters of one training step (Kingma & Ba 2015); the step
 * count t lives in the handle and starts at 1 on the first step. */
typedef struct {
  float lr, beta1, beta2, eps;
} qtree_adam;

/* Device bytes a qtree_mlp needs to train on batches of up to max_batch
 * samples (0: inference only).  EINVAL if max_batch < 0 or > 2^24. */
qtree_status qtree_mlp_workspace_size(int64_t max_batch, size_t *bytes);

/* Lay the network out in `workspace` (device, >= qtree_mlp_workspace_size
 * bytes, 256-byte aligned) and upload params_host (FP32 [133633]).
 * lo, hi: host float[6], the training box (lo <= hi); out_scale: s;
 * act_terms: 1 or 2; baseline: 0 or 1 (base(x) above; 1 needs sigma > 0,
 * T > 0 and S0/K > 0 inside the box).  Synchronous.  EINVAL on a bad
 * argument, ENOMEM if the workspace is too small. */
qtree_status qtree_mlp_create(const float *params_host, const float *lo, const float *hi,
                              float out_scale, int32_t act_terms, int32_t baseline,
                              int64_t max_batch, void *workspace, size_t workspace_bytes,
                              qtree_mlp **out);
void qtree_mlp_destroy(qtree_mlp *mlp);

/* Copy the FP32 master parameters to the host (synchronous). */
qtree_status qtree_mlp_get_params(const qtree_mlp *mlp, float *params_host);
/* Replace the parameters (synchronous); Adam moments and the step count
 * restart at zero. */
qtree_status qtree_mlp_set_params(qtree_mlp *mlp, const float *params_host);

/* Inference: y[b] = network(x[b]) for x: device float[B][6] (raw
 * parameters), y: device float[B]; in_range (device uint8[B] or NULL) gets
 * 1 where lo <= x[b] <= hi in every slot.  Needs no training buffers; any
 * B >= 0 (B = 0 does nothing). */
qtree_status qtree_mlp_forward(const qtree_mlp *mlp, const float *x, int64_t B, float *y,
                               uint8_t *in_range, void *stream);

/* Loss L = sum_b w_b (y_b - t_b)^2 / B over the batch rows idx[0..B) of the
 * training set (x: device float[rows][6], t, w: device float[rows]; w NULL
 * = all ones; idx: device int32[B] row indices, or NULL for rows 0..B-1)
 * and its gradient with respect to the parameters (the roundings of the
 * forward pass taken as the identity).  grad: device float[133633] or NULL,
 * loss: device float[1] or NULL.  1 <= B <= max_batch. */
qtree_status qtree_mlp_grad(qtree_mlp *mlp, const float *x, const float *t, const float *w,
                            const int32_t *idx, int64_t B, float *grad, float *loss,
                            void *stream);

/* qtree_mlp_grad followed by one Adam step on the master parameters and
 * the refresh of their BF16 copies. */
qtree_status qtree_mlp_train_step(qtree_mlp *mlp, const float *x, const float *t, const float *w,
                                  const int32_t *idx, int64_t B, const qtree_adam *opt,
                                  float *loss, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* QTREE_MLP_H */
