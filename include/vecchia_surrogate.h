/*
 * vecchia_surrogate.h -- C ABI of the learned surrogate of the Vecchia
 * conditional densities (MI355X / gfx950), built beside the exact path of
 * vecchia.h.
 *
 * Every factor of the Vecchia approximation (Section 2.1, Eq. 3) is a
 * Gaussian conditional density N(b' y_s, v) whose kriging weights b and
 * variance v depend only on the neighbourhood's geometry in range units,
 * the smoothness and the nugget ratio.  A small MLP learns that map from
 * neighbourhoods the exact FP64 kernel solved (vec_kriging_weights) and
 * then stands in for the factorisation: for a served observation the
 * log-likelihood terms of Algorithm 1 are formed in FP64 from the predicted
 * b and log v; observations the network does not serve are handed back for
 * the exact path (vec_loglik_sums_at).  Scope: the 2-D isotropic family,
 * m = VEC_SURROGATE_M neighbours.
 *
 * Network: VEC_MLP_IN inputs -> three hidden layers of VEC_MLP_HIDDEN
 * units with SiLU -> VEC_MLP_OUT outputs.  Inputs of observation i: the m
 * neighbours' offsets (x_s - x_i) / rho in NNarray column order (2m
 * values), nu, tau2, zeros.  Outputs: b_1..b_m, then log(v / sigma2)
 * affinely scaled (value = output * lv_scale + lv_shift), then one unused.
 * Parameters, in this order, W row-major as W[out][in]:
 *   W0[H][IN] b0[H] W1[H][H] b1[H] W2[H][H] b2[H] W3[OUT][H] b3[OUT]
 * held twice by the caller: FP32 (biases, optimiser state) and BF16 (the
 * weights the matrix cores read); vec_mlp_to_bf16 and vec_mlp_adam keep
 * the BF16 copy in step.  BF16 arrays are passed as uint16_t (raw bits).
 *
 * Conventions (pointers, streams, errors, status) as in vecchia.h.  Row
 * counts of the network calls are multiples of 32 (pad with zero rows).
 */
#ifndef VECCHIA_SURROGATE_H
#define VECCHIA_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "vecchia.h"

#ifdef __cplusplus
extern "C" {
#endif

#define VEC_SURROGATE_M 30
#define VEC_MLP_IN 64
#define VEC_MLP_HIDDEN 256
#define VEC_MLP_OUT 32

/* Number of network parameters (FP32 and BF16 arrays hold this many). */
int64_t vec_mlp_param_count(void);

/* Device workspace bytes for `rows` rows of vec_mlp_forward (training = 0:
 * a copy of the weights, whatever the row count) or vec_mlp_loss_grad
 * (training != 0); 0 if rows is invalid. */
size_t vec_mlp_workspace_bytes(int64_t rows, int32_t training);

/* y[rows][OUT] (FP32) = network(x[rows][IN] (BF16)): the weights are copied
 * into the workspace in the order the matrix-core operands take them, then
 * the whole network runs in one launch.  rows: a positive multiple of 32, at
 * most 2^24.  x, params, y and workspace 16-byte aligned (VEC_EINVAL
 * otherwise). */
int vec_mlp_forward(int64_t rows, const uint16_t* x, const float* params,
                    const uint16_t* params_bf16, float* y, void* workspace,
                    size_t workspace_bytes, void* stream);

/* One forward and backward pass of the weighted squared error
 *   loss = scale * sum_r sum_c colw[c] (y[r][c] - targets[r][c])^2
 * (targets FP32 [rows][OUT], colw FP32 [OUT]): grad[param_count] (FP32)
 * and *loss (device double) are overwritten.  Weight gradients are summed
 * over rows with FP32 atomics (order not fixed). */
int vec_mlp_loss_grad(int64_t rows, const uint16_t* x, const float* targets, const float* colw,
                      float scale, const float* params, const uint16_t* params_bf16, float* grad,
                      double* loss, void* workspace, size_t workspace_bytes, void* stream);

/* One Adam step (bias-corrected, step >= 1) on the FP32 parameters with
 * moments m1, m2 (FP32, zero before the first step); the BF16 copy is
 * rewritten. */
int vec_mlp_adam(const float* grad, float* params, uint16_t* params_bf16, float* m1, float* m2,
                 int32_t step, float lr, float beta1, float beta2, float eps, void* stream);

/* params_bf16 = BF16(params), round to nearest even. */
int vec_mlp_to_bf16(const float* params, uint16_t* params_bf16, void* stream);

/* Network inputs of observations [i0, i1) of a 2-D isotropic problem with
 * m = VEC_SURROGATE_M: features[(i - i0)][IN] (BF16).  flag[(i - i0)] (may
 * be NULL) = 1 for observations the network must not serve: i < m, a
 * malformed NNarray row, or a neighbour offset whose scaled length lies
 * outside [dist_lo, dist_hi] (the geometry the network was trained on).
 * features 16-byte aligned (VEC_EINVAL otherwise). */
int vec_surrogate_features(const vec_problem* pb, const double* locs, const int32_t* NNarray,
                           const double* covparms, int64_t i0, int64_t i1, float dist_lo,
                           float dist_hi, uint16_t* features, uint8_t* flag, void* stream);

/* Device workspace bytes of vec_surrogate_sums. */
size_t vec_surrogate_workspace_bytes(const vec_problem* pb);

/* FP64 sums of vec_loglik (logdet, ySy, XSX, ySX; 2 + p*p + p doubles) over
 * the observations of [i0, i1) that the network serves, from its outputs
 * pred[(i - i0)][OUT] (16-byte aligned, VEC_EINVAL otherwise): with
 * b = pred[..][0..m-1] and
 * lv = pred[..][m] * lv_scale + lv_shift, the residuals are
 * e_y = y_i - b.y_s and e_X = X_i - b.X_s and the variance is
 * v = sigma2 exp(lv).  An observation is handed back instead (its index
 * appended at back[atomic (*nback)++], order not fixed) if flag marks it,
 * if it has fewer than m neighbours or a malformed NNarray row, if lv lies
 * outside [log tau2, log(1 + tau2)] widened by lv_slack (no conditional
 * variance of the model lies outside that interval), or if lv < lv_floor.
 * The floor is the accuracy gate: an error d in the weights changes the
 * term by about (d' Sigma_s d) / (2 v), so neighbourhoods with a small
 * conditional variance (strongly correlated, little nugget) need weights
 * far more accurate than BF16 gives and are better handed back.
 * raw is overwritten (accumulate = 0) or added to (accumulate != 0); the
 * caller zeroes *nback and sizes back for every observation of the calls
 * that share it. */
int vec_surrogate_sums(const vec_problem* pb, const int32_t* NNarray, const double* y,
                       const double* X, const double* covparms, int64_t i0, int64_t i1,
                       const float* pred, const uint8_t* flag, float lv_scale, float lv_shift,
                       float lv_slack, float lv_floor, double* raw, int32_t accumulate,
                       int32_t* back, uint32_t* nback, void* workspace, size_t workspace_bytes,
                       void* stream);

#ifdef __cplusplus
}
#endif

#endif /* VECCHIA_SURROGATE_H */
