/*
 * gsr_scorer.h - learned candidate scorer of libgsr (MI355X, gfx950).
 *
 * The brute-force search of Sec. III-C1 renders every candidate pose and
 * compares it with the query by NCC (Eq. 10); Sec. IV shortens that search by
 * scoring only part of the candidates. This scorer is a pruning step before
 * the full-resolution comparison: a small convolutional network maps a
 * low-resolution render of a candidate and the equally pooled query to a
 * predicted NCC, so that only the best-predicted candidates are rendered at full
 * resolution and scored by the exact NCC (which keeps the final say). It is trained
 * on pairs that the renderer itself produces, labelled with their full-resolution
 * NCC, by the kernels below (forward, backward, AdamW) on the GPU.
 *
 * Network input of one candidate: [h][w][2] bfloat16 (raw uint16 bits), channel
 * 0 = the BT.601 grey of the render, channel 1 = the query's pooled grey, each
 * standardised to zero mean and unit variance over its pixels (a constant image
 * gives zeros). Network, on NHWC activations with 3x3 zero-padded convolutions:
 *   conv 2->32 stride 2, ReLU; conv 32->64, ReLU; conv 64->64 stride 2, ReLU;
 *   conv 64->128, ReLU; conv 128->128 stride 2, ReLU; global average pool;
 *   linear 128->128, ReLU; linear 128->1 = predicted score.
 * Output size of a stride-s convolution over n pixels: (n - 1) / s + 1.
 * Convolution weights and activations are bfloat16 (round to nearest even), with
 * float32 sums on the matrix cores; pooling, linear layers, loss and optimiser are
 * float32. Parameters are one flat float32 vector of gsr_scorer_param_count()
 * entries: per convolution W[c_out][3][3][c_in] then b[c_out]; then W1[128][128]
 * (out, in), b1[128], w2[128], b2[1].
 *
 * Memory: *_dev pointers are caller-owned device memory; the scorer owns its
 * parameters, optimiser state and activation buffers (sized for max_batch). All
 * calls enqueue on the context's stream and return without waiting. A scorer
 * belongs to the context it was created on and must be destroyed before it;
 * calls on one scorer must not overlap.
 */
#ifndef GSR_SCORER_H
#define GSR_SCORER_H

#include <stdint.h>

#include "gsr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gsr_scorer gsr_scorer;

/* AdamW (decoupled weight decay); the decay applies to weights, not biases. */
typedef struct {
    float lr, beta1, beta2, eps, weight_decay;
} gsr_adamw;

/* Number of float32 parameters (294,113). */
int64_t gsr_scorer_param_count(void);

/* Scorer for inputs of height x width pixels (1..4096 each) and batches of up to
 * max_batch candidates (1..65535). Parameters start at zero: set them with
 * gsr_scorer_set_params. GSR_ENOMEM if the buffers do not fit. */
int gsr_scorer_create(gsr_ctx *ctx, int32_t height, int32_t width, int32_t max_batch, gsr_scorer **out);
/* Waits for the context's stream and frees the scorer. */
int gsr_scorer_destroy(gsr_scorer *s);

/* Copy the flat float32 parameters in (and reset the optimiser state and step
 * count) or out. params_dev: [gsr_scorer_param_count()] device memory. */
int gsr_scorer_set_params(gsr_scorer *s, const float *params_dev);
int gsr_scorer_get_params(gsr_scorer *s, float *params_dev);

/* grey_dev[i] = factor x factor mean pool of the BT.601 grey of rgb_dev[i]
 * ([n][3][height][width] float32 planar; height and width multiples of factor),
 * giving [n][height/factor][width/factor] float32. Used for the query. */
int gsr_pool_grey(gsr_ctx *ctx, const float *rgb_dev, int32_t n, int32_t height, int32_t width, int32_t factor,
                  float *grey_dev);

/* Network inputs x_dev [n][h][w][2] (bf16 bits) from n renders renders_dev
 * [n][3][h][w] float32 planar and the pooled query query_grey_dev [h][w]. */
int gsr_scorer_inputs(gsr_scorer *s, const float *renders_dev, int32_t n, const float *query_grey_dev,
                      uint16_t *x_dev);

/* Predicted scores [n] of n inputs x_dev [n][h][w][2] (4-byte aligned). */
int gsr_scorer_forward(gsr_scorer *s, const uint16_t *x_dev, int32_t n, float *scores_dev);

/* Loss = mean over the n candidates of (score - label)^2 and its gradient with
 * respect to the flat parameters, at the current parameters; nothing is updated.
 * labels_dev [n]; loss_dev [1] or NULL; grads_dev [gsr_scorer_param_count()]. */
int gsr_scorer_backward(gsr_scorer *s, const uint16_t *x_dev, const float *labels_dev, int32_t n, float *loss_dev,
                        float *grads_dev);

/* One AdamW step with the gradient grads_dev [gsr_scorer_param_count()]:
 *   m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 *   p = p - lr wd p (weights only) - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps),
 * t = steps taken since gsr_scorer_set_params, counting this one. */
int gsr_scorer_adamw(gsr_scorer *s, const float *grads_dev, const gsr_adamw *opt);

/* gsr_scorer_backward into the scorer's own gradient buffer, then
 * gsr_scorer_adamw with it. loss_dev [1] or NULL. */
int gsr_scorer_train_step(gsr_scorer *s, const uint16_t *x_dev, const float *labels_dev, int32_t n,
                          const gsr_adamw *opt, float *loss_dev);

/* Pruned candidate search. Every candidate pose is rendered at the low
 * resolution cam_low (batch candidates at a time; 0 = automatic) and given a
 * predicted score: the scorer's output, or with scorer == NULL the NCC of the
 * low-resolution render against the pooled query (the same pruning without the
 * network). The k candidates with the best predictions (ties: lower index) are
 * rendered at full resolution (cam) and scored by NCC against the query
 * (Eq. 10), which decides among them. The full-resolution image must be f times
 * the low-resolution one in both directions (integer f); cam_low is normally cam
 * with focal lengths and principal point divided by f. One host wait at the end
 * (and one per render, see gsr_render_cfg.pair_capacity).
 *   poses_dev [P,3,4] float32 world-to-camera, 1 <= k <= P <= 8192
 *   query_dev [3,H,W] float32 full-resolution query
 *   pred_dev  [P] float32 output: predicted score of every candidate
 *   top_dev   [k] int32 output: the kept candidates, best prediction first
 *   ncc_dev   [k] float32 output: their full-resolution NCC
 *   best, best_score (host): the kept candidate with the highest NCC (ties: lower
 *   candidate index) and that NCC.
 * The scorer, if given, must belong to ctx and take cam_low's image size. */
int gsr_search_pruned(gsr_ctx *ctx, gsr_scorer *scorer, const gsr_submap *sm, const gsr_camera *cam,
                      const gsr_camera *cam_low, const float *poses_dev, int32_t n_poses, int32_t batch,
                      const float *query_dev, int32_t k, const gsr_render_cfg *cfg, float *pred_dev, int32_t *top_dev,
                      float *ncc_dev, int32_t *best, float *best_score);

#ifdef __cplusplus
}
#endif

#endif /* GSR_SCORER_H */
