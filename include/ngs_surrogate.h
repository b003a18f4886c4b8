/* ngs_surrogate.h -- learned view scorer of libngs (extends ngs.h).
 *
 * Not part of arXiv 2602.08266: an addition that predicts a candidate view's next-best-view
 * score (Eq. 11 of the paper, as computed exactly by ngs_score_batch) from four low-resolution
 * rendered feature maps (depth, final transmittance, argmax object id, and the ray average of
 * a per-Gaussian weight such as confidence x novelty; ngs_sur_render_features). The exact
 * information gain makes the final choice: callers re-score the surrogate's best candidates
 * with ngs_score_batch.
 *
 * Network (fixed): four 3x3 convolutions, stride 2, padding 1, ReLU
 * (4 -> 32 -> 64 -> 128 -> 128 channels; 60x80 -> 30x40 -> 15x20 -> 8x10 -> 4x5), global
 * average pool, fully connected 128 -> 128 (ReLU) -> 1. Every convolution and fully connected
 * layer runs as a GEMM on BF16 operands with FP32 accumulation on the matrix cores; weights
 * are kept in FP32 (master copy) and BF16 (operand copy).
 *
 * Layouts: activations and inputs are channel-major, x [4][B][60][80] FP32. Layer l
 * (0..3 convolutions, 4..5 fully connected) has weight w[l] [out][in * 9] (convolutions,
 * index in * 9 + kh * 3 + kw) or [out][in], bias b[l] [out]. All pointers are caller-owned
 * device memory; every call is stream-ordered and does not synchronise. */
#ifndef NGS_SURROGATE_H
#define NGS_SURROGATE_H

#include "ngs.h"

#ifdef __cplusplus
extern "C" {
#endif

#define NGS_SUR_LAYERS 6
#define NGS_SUR_WIDTH 128
#define NGS_SUR_IN_C 4
#define NGS_SUR_IN_H 60
#define NGS_SUR_IN_W 80

typedef struct {
  float* w[NGS_SUR_LAYERS];          /* FP32 weights (gradients, Adam moments: same shapes) */
  float* b[NGS_SUR_LAYERS];          /* FP32 biases */
  uint16_t* w_bf16[NGS_SUR_LAYERS];  /* BF16 copies of w (NULL in gradient / moment sets) */
} ngs_sur_params;

/* Scratch bytes of ngs_sur_forward / ngs_sur_backward for a batch of `batch` views. */
ngs_status ngs_sur_workspace_size(int32_t batch, size_t* bytes);

/* Writes the BF16 operand copies from the FP32 weights. */
ngs_status ngs_sur_sync_bf16(ngs_ctx* ctx, const ngs_sur_params* params, void* stream);

/* pred [batch] = network(x). Keeps the activations the backward pass needs in ws, laid out
 * (for this batch) as: for each convolution l = 0..3 in turn, its im2col operand col_l (BF16
 * [ci * 9][batch * ho * wo]) and its output act_l after the ReLU (FP32 [co][batch * ho * wo]);
 * then the pooled activations (FP32 [128][batch]) and their BF16 copy, the hidden layer after
 * its ReLU (FP32 [128][batch]) and its BF16 copy; every region starts on a 256-byte boundary. */
ngs_status ngs_sur_forward(ngs_ctx* ctx, const ngs_sur_params* params, const float* x, int32_t batch,
                           float* pred, void* ws, size_t ws_bytes, void* stream);

/* Gradients of a loss with d loss / d pred = dpred [batch] w.r.t. every weight and bias
 * (written to grads->w, grads->b), using the activations of the last ngs_sur_forward on the
 * same ws, params and x. */
ngs_status ngs_sur_backward(ngs_ctx* ctx, const ngs_sur_params* params, const float* x, int32_t batch,
                            const float* dpred, ngs_sur_params* grads, void* ws, size_t ws_bytes, void* stream);

/* Mean squared error: loss[0] = mean (pred - target)^2 (loss may be NULL), dpred = 2 (pred -
 * target) / batch. */
ngs_status ngs_sur_mse(ngs_ctx* ctx, const float* pred, const float* target, int32_t batch, float* dpred,
                       float* loss, void* stream);

/* One Adam step (bias-corrected, step >= 1) on every weight and bias of params with gradients
 * g and moments m, v; refreshes the BF16 copies. */
ngs_status ngs_sur_adam(ngs_ctx* ctx, ngs_sur_params* params, const ngs_sur_params* g, ngs_sur_params* m,
                        ngs_sur_params* v, float lr, float beta1, float beta2, float eps, int32_t step,
                        void* stream);

/* Input channels of view `index` (0 <= index < batch) from its width x height ngs_render
 * output (depth, t_final, argmax_id, mean_conf): depth / depth_scale, t_final, argmax id / k,
 * mean confidence, written to x [4][batch][height][width]. */
ngs_status ngs_sur_features(ngs_ctx* ctx, const ngs_image* img, int32_t width, int32_t height, int32_t k,
                            float depth_scale, float* x, int32_t batch, int32_t index, void* stream);

/* Per-Gaussian novelty against a training store (device, out [n] FP32):
 * out[g] = c_g * (1/3) sum_f exp(-(logdet H_T,g,f - d_f ln lambda) / d_f) over the outputs
 * f = rgb, depth, object (d_f = 14, 11, 11 + k; Eq. 9 blocks with the prior lambda I), i.e. the
 * confidence of Eq. 7 / 12 times the mean reciprocal geometric-mean eigenvalue of H_T / lambda:
 * c_g for a Gaussian no training view touched (or h NULL), smaller the better it is observed.
 * lambda_prior must be the one the store was built with. The scene must be prepared.
 * An input the surrogate's feature render averages (not part of the paper's method). */
ngs_status ngs_sur_novelty(ngs_ctx* ctx, const ngs_scene* scene, const ngs_hessian* h, float lambda_prior,
                           float* out, void* stream);

/* Feature maps of n_views candidates (every camera 80 x 60) in one call: per view, projection,
 * binning and compositing (as ngs_project, ngs_bin_sort, ngs_render) and the four input
 * channels into x [4][n_views][60][80] (as ngs_sur_features, depth / depth_scale). With
 * weight (device [n], may be NULL) the fourth channel averages weight[g] along each ray
 * where ngs_render averages kappa (e.g. the output of ngs_sur_novelty). Views go in groups
 * of dims->views_in_flight (default 8, at most 32): each view of a group is projected and
 * binned on its own context stream, then one render launch composites the whole group; no
 * host synchronisation except one at the end. The scene must be prepared. ws:
 * ngs_workspace_size(4, dims) bytes. NGS_CAPACITY if a view has more pairs than
 * dims->max_pairs. */
ngs_status ngs_sur_render_features(ngs_ctx* ctx, const ngs_scene* scene, const ngs_camera* cams, int32_t n_views,
                                   const ngs_raster_params* rp, const float* weight, float depth_scale, float* x,
                                   const ngs_dims* dims, void* ws, size_t ws_bytes, void* stream);

/* The surrogate-guided choice with the exact information gain as judge: ranks the n_views
 * candidates (host camera array) by the network's predictions pred (device FP32 [n_views],
 * e.g. ngs_sur_forward over the maps of ngs_sur_render_features), re-scores the best
 * `rescore` of them exactly (as ngs_score_batch with h, normalisers, rp, ig, dims and ws;
 * Eq. 5, 10, 11) and returns in *best (host) the index into cams of the exact argmax among
 * them. chosen (host int32 [rescore]) receives the re-scored candidates' indices by descending
 * prediction (lower index first on ties, a prediction that is not a number last); scores
 * (device FP32 [rescore][4]) and ig_raw (device FP64 [rescore][3]) their exact scores and
 * gains, in that order. rescore > n_views re-scores every candidate. Syncs. Status as
 * ngs_score_batch. */
ngs_status ngs_sur_pick(ngs_ctx* ctx, const ngs_scene* scene, ngs_hessian* h, const double* normalisers,
                        const ngs_camera* cams, int32_t n_views, const float* pred, int32_t rescore,
                        const ngs_raster_params* rp, const ngs_ig_params* ig, int32_t* chosen, float* scores,
                        double* ig_raw, int32_t* best, int64_t* stats, const ngs_dims* dims, void* ws,
                        size_t ws_bytes, void* stream);

/* c [m][n] = op(a) op(b) + beta c with BF16 a, b (raw 16-bit words) and FP32 c on the matrix
 * cores. op(a) = a [m][k] (lda) or, with trans_a, a^T of a [k][m]; op(b) = b [k][n] (ldb) or,
 * with trans_b, b^T of b [n][k]. The kernel every surrogate layer uses. */
ngs_status ngs_gemm_bf16(ngs_ctx* ctx, int32_t trans_a, int32_t trans_b, int32_t m, int32_t n, int32_t k,
                         const uint16_t* a, int32_t lda, const uint16_t* b, int32_t ldb, float* c, int32_t ldc,
                         float beta, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NGS_SURROGATE_H */
