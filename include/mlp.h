/*
 * mlp.h -- learned proposal for batched BOS (part of libcorr).
 *
 * A small multilayer perceptron maps a region pair's summary to the maxima
 * BOS searches for (Sec. 3.1) and a proposed location; its prediction seeds
 * the sampler through bos_set_prior. The paper names a network trained to
 * predict correlation values as future work (Sec. 7); here it is trained on
 * records the method itself produces (exhaustive / BOS maxima).
 *
 * Network: x (n_in) -> silu(x W1 + b1) -> silu(. W2 + b2) -> . W3 + b3 (n_out),
 * silu(z) = z / (1 + e^-z), weights W [in][out] row-major. Parameters are
 * FP32 master values; forward and backward use their BF16 roundings with FP32
 * arithmetic. Training minimises the weighted mean squared error
 * sum_{b,o} w_o (y_bo - t_bo)^2 / (B n_out) with AdamW (beta1 0.9,
 * beta2 0.999, eps 1e-8, decoupled weight decay). Every reduction runs in a
 * fixed order, so results are bitwise reproducible.
 * Flat parameter order: W1, b1, W2, b2, W3, b3.
 */
#ifndef CORR_MLP_H
#define CORR_MLP_H

#include <stdint.h>

#include "corr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct prop_mlp prop_mlp;

/* Create a network (n_in, n_hidden <= 1024, n_out <= 64, batch size up to
 * 4096 per call); weights Glorot-uniform from Philox4x64-10 with `seed`,
 * biases 0, AdamW moments 0. */
int prop_mlp_create(corr_ctx* ctx, int32_t n_in, int32_t n_hidden, int32_t n_out, uint64_t seed, prop_mlp** out);

/* Number of parameters (FP32 master values). */
int prop_mlp_num_params(prop_mlp* m, int64_t* n);

/* Copy the FP32 master parameters out of / into the network (HOST arrays of
 * prop_mlp_num_params floats). Setting resets nothing else. */
int prop_mlp_get_params(prop_mlp* m, float* params);
int prop_mlp_set_params(prop_mlp* m, const float* params);

/* Forward pass: x device [B][n_in] -> y device [B][n_out]. */
int prop_mlp_forward(prop_mlp* m, const float* x, int32_t B, float* y, corr_stream_t stream);

/* One training step on a batch: forward, weighted-MSE gradient (loss_w HOST
 * [n_out] or NULL for all ones), backward, AdamW update of the master
 * parameters with learning rate lr and weight decay wd. loss_out (HOST,
 * nullable; then the call synchronises) receives the batch loss before the
 * update. */
int prop_mlp_train_step(prop_mlp* m, const float* x, const float* target, const float* loss_w, int32_t B, float lr,
                        float wd, float* loss_out, corr_stream_t stream);

/* Gradient of the last training step (HOST, prop_mlp_num_params floats). */
int prop_mlp_get_grads(prop_mlp* m, float* grads);

/* Free the network. NULL is allowed. */
void prop_mlp_destroy(prop_mlp* m);

/*
 * Inputs of the proposal network for region pairs of one field A (device
 * x_out [n_pairs][2 (4 n_hot + 5) + n_hot^2], row-major).
 *   zhat_p   centred, unit-norm member vector of grid point p (0 if constant)
 *   s(p)     mean of zhat_p . zhat_q over the grid points q = p +- D e_x,
 *            p +- D e_y, p +- D e_z that lie inside the grid (0 if none)
 *   picks    per region, n_hot points: pick i is the first point (local
 *            x-fastest order) with the largest s among the region's points
 *            whose Chebyshev distance to every earlier pick exceeds r_nms;
 *            when none qualifies the previous pick is repeated
 *   region   per pick: s, local (x, y, z) / (extent - 1) (0 for extent 1);
 *            then the region mean of the per-point means, the region mean of
 *            the per-point population standard deviations, and the region
 *            centre divided by the grid extent (x, y, z)
 *   pair     region values of a, of b, then |zhat_{a_i} . zhat_{b_j}|,
 *            i, j < n_hot, i outer.
 * region_pairs is a HOST array [n_pairs][2] of indices into `regions`.
 * hot_out (device [n_regions][n_hot] global point indices) may be NULL.
 * 1 <= n_hot <= 8, D >= 1, r_nms >= 0, M >= 2. Per-point statistics are
 * accumulated in FP64, dot products in FP32; every sum runs in a fixed
 * order. Synchronises `stream` (the pair list is staged from the host).
 */
int corr_proposal_inputs(corr_ctx* ctx, const corr_field* A, const corr_region* regions, int32_t n_regions,
                         const int32_t* region_pairs, int32_t n_pairs, int32_t n_hot, int32_t D, int32_t r_nms,
                         float* x_out, int32_t* hot_out, corr_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* CORR_MLP_H */
