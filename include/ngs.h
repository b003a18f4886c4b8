/* ngs.h -- C ABI of the MI355X (gfx950) next-best-view scorer for object-aware
 * 3D Gaussian Splatting (arXiv 2602.08266).
 *
 * The library renders colour, depth and the object vector of a Gaussian map for
 * candidate camera poses (tile-based splatting, Sec. III-A, Eq. 1-2) and scores each
 * pose by the confidence-weighted, block-diagonal log-det information gain
 * (Sec. III-B, Eq. 5-11), normalised per output by the training views.
 *
 * Conventions
 *  - Every function returns ngs_status; no C++ exception crosses the ABI. On error the
 *    outputs are unspecified and the context stays usable.
 *  - Array arguments are caller-owned, contiguous DEVICE pointers unless marked
 *    "host". The library never frees, retains or reallocates caller memory.
 *  - All work is enqueued on the caller's stream (hipStream_t passed as void*; NULL is
 *    the default stream). Outputs are valid after the stream is synchronised.
 *    Functions that must read a device count back (marked "syncs") synchronise the
 *    stream before returning.
 *  - Float arrays are FP32 structure-of-arrays: "[3][n]" means three planes of n.
 *    Per-output information-gain sums are FP64.
 *  - One context per host thread; a context is bound to one device.
 */
#ifndef NGS_H
#define NGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t ngs_status;
#define NGS_OK 0
#define NGS_INVALID_ARG (-1)      /* NULL where a pointer is required, negative size ... */
#define NGS_CAPACITY (-2)         /* an output buffer is too small; the needed size is reported */
#define NGS_WORKSPACE_TOO_SMALL (-3)
#define NGS_HIP_ERROR (-4)        /* a HIP runtime call failed; see ngs_last_hip_error */
#define NGS_DEGENERATE (-5)       /* an enabled Eq. 10 normaliser is not positive */
#define NGS_UNSUPPORTED (-6)      /* e.g. k > 64, tile != 16, more than 4096 tiles */

#define NGS_MAX_K 64
#define NGS_MAX_TILES 4096

/* Output bits of ngs_ig_params.outputs (Sec. III-B.3). */
#define NGS_OUT_RGB 1u
#define NGS_OUT_DEPTH 2u
#define NGS_OUT_OBJ 4u

/* ngs_ig_params.mode */
#define NGS_MODE_SCORE 0          /* IG_f(T, c) of one candidate view (Eq. 5) */
#define NGS_MODE_ACCUMULATE 1     /* add c_g * A_t,g of a training view into H_T (Eq. 9) */

typedef struct ngs_ctx ngs_ctx;

/* Gaussian map (Sec. III-A.1): mean mu, log-scale, raw quaternion (w, x, y, z), opacity
 * logit, SH degree-0 colour and object logits o of length k = n_objects + 1 (channel 0 is
 * the background). The derived arrays are caller-allocated and written by
 * ngs_prepare_scene: prob = softmax(o) row-major [n][k]; opacity = sigmoid(logit);
 * kappa = max_k prob; conf = c_g of Eq. 7 (or Eq. 12 for a target); label = argmax_k
 * prob (lowest k on ties). */
typedef struct {
  int32_t n, k;
  const float* mean;           /* [3][n] */
  const float* log_scale;      /* [3][n] */
  const float* rot;            /* [4][n] */
  const float* opacity_logit;  /* [n] */
  const float* rgb;            /* [3][n] */
  const float* obj_logit;      /* [k][n] */
  float* prob;                 /* [n][k] derived */
  float* opacity;              /* [n] derived */
  float* kappa;                /* [n] derived */
  float* conf;                 /* [n] derived */
  int32_t* label;              /* [n] derived */
  double* cov3;                /* [9][n] derived, may be NULL: the 3D covariance
                                  Sigma3 = Rg diag(s^2) Rg^T (row-major 3x3, FP64, the
                                  projection's own operation order), so that ngs_project
                                  reads it instead of recomputing it for every view */
} ngs_scene;

/* Pinhole camera: world -> camera rotation R (row-major) and translation t; OpenCV axes
 * (x right, y down, z forward); focal lengths and principal point in pixels. */
typedef struct {
  float R[9];
  float t[3];
  float fx, fy, cx, cy;
  int32_t width, height;
} ngs_camera;

/* Rasterizer constants of the 3DGS pipeline the paper follows (Sec. IV-A.2):
 * tile = 16, z_near = 0.05, eps2d = 0.3, cutoff_q = 9, alpha_min = 1/255,
 * alpha_max = 0.99, t_min = 1e-4. */
typedef struct {
  int32_t tile;
  float z_near, eps2d, cutoff_q, alpha_min, alpha_max, t_min;
} ngs_raster_params;

/* Information-gain constants: Eq. 7 exponents (0.3, 0.3) and Eq. 11 weights (10, 1)
 * from Sec. IV-A.2; lambda_prior adds lambda*I to every block of H (a reading: the
 * paper is silent on regularisation); target_id < 0 scores the whole scene (Eq. 7),
 * otherwise Eq. 12 for that object; conf_on_train = 1 weights training views by c_g
 * too (Eq. 9 read for every view); obj_eq2 = 1 differentiates O of Eq. 2 (else O').
 * criterion selects f (Sec. III-B): 0 = log det H (Eq. 6, the paper's choice); 1 = the
 * trace-based f(V) = trace(H_V^-1)^-1 on the same block-diagonal H. With 1 the raw gain of
 * a view is the covariance-trace reduction R_f = sum_g [trace(H_T,g^-1) -
 * trace((H_T,g + c_g A_g)^-1)] and ngs_score_batch turns it into f(T + c) - f(T) =
 * R / (S (S - R)) with trace_total[f] = S = sum over all n Gaussians of trace(H_T,g^-1)
 * (n - stored slots times l_f / lambda for Gaussians without a stored block); the
 * normalisers must then be means of that converted quantity over the training views.
 * Ablation switches of the paper's Table III: the object output (bit 2 of outputs), the
 * confidence (alpha_obj = alpha_opa = 0 gives c_g = 1, or the target indicator with
 * Eq. 12), and the Eq. 10 scaling (normalisers 1 with fixed beta weights). */
typedef struct {
  float lambda_prior, alpha_obj, alpha_opa, beta_d, beta_o;
  int32_t target_id;
  uint32_t outputs;
  int32_t conf_on_train;
  int32_t obj_eq2;
  int32_t mode;
  int32_t criterion;
  double trace_total[3];
} ngs_ig_params;

/* Per-view projection (one entry per Gaussian). rect holds each Gaussian's inclusive
 * tile bounds (x0, y0, x1, y1) together (8 bytes, 8-byte aligned; a culled Gaussian has
 * (0, 0, -1, -1)); count = number of tiles (0: culled). zkey = bits of float32(Z).
 * splat (16-byte aligned) packs what the information walk reads of an entry into one
 * record per Gaussian: [n][8] = 2D mean x, y, conic xx, xy, yy, opacity, half-extents x, y
 * of the ellipse q <= cutoff_q (widened for rounding). ngs_project writes it when it is not
 * NULL (the scene must then be prepared: it copies the opacity); ngs_info_gain reads it. */
typedef struct {
  float* mean2d;    /* [2][n] */
  float* conic;     /* [3][n] Q = Sigma2^-1: xx, xy, yy */
  float* depth;     /* [n] camera-space Z */
  uint32_t* zkey;   /* [n] */
  int16_t* rect;    /* [n][4] */
  uint32_t* count;  /* [n] */
  float* splat;     /* [n][8] or NULL */
} ngs_projected;

/* Per-view tile lists: (tile, depth, gid)-sorted Gaussian ids and per-tile ranges.
 * keys (optional) = (tile << 32) | zkey. n_pairs is a device scalar. An empty tile has
 * start = end = the number of pairs in lower tiles. */
typedef struct {
  uint64_t* keys;     /* [capacity] or NULL */
  uint32_t* gids;     /* [capacity] */
  int64_t capacity;
  int64_t* n_pairs;   /* [1] */
  uint32_t* ranges;   /* [2][tiles]: start, end */
} ngs_tile_lists;

/* Rendered images, planes of H x W. Optional outputs may be NULL. */
typedef struct {
  float* rgb;          /* [3][H][W] */
  float* depth;        /* [H][W] sum of Z alpha T (unnormalised, background 0) */
  float* obj;          /* [k][H][W] O of Eq. 2, or NULL */
  float* t_final;      /* [H][W] */
  float* mean_conf;    /* [H][W] sum kappa alpha T / (1 - T_final), or NULL */
  int32_t* argmax_id;  /* [H][W] argmax_k O_k (lowest k on ties) */
  int32_t* n_contrib;  /* [H][W] or NULL */
} ngs_image;

/* Training information H_T (Eq. 9 with prior lambda*I), stored only for Gaussians
 * that a training view touched; every other Gaussian has H_T = lambda*I. Slot-major, FP64,
 * each slot's block contiguous:
 *   h_rgb[slot * 105 + e]  packed upper triangle, row-major, of the 14 x 14 RGB block;
 *   h_d[slot * 66 + e]     the same for the 11 x 11 depth block;
 *   h_o[slot * (68 + 12k) + e]  the (11+k) x (11+k) object block in factored form: for
 *     softmax probabilities p and S = diag(p) - p p^T every such block (and every sum of
 *     them plus lambda*I) is [[G, E S], [S E^T, lambda I + tau S S]]; stored are G (packed
 *     upper 11 x 11, e < 66), tau (e = 66), lambda (e = 67), E (11 x k row-major,
 *     e = 68 + r k + c) and p (e = 68 + 11k + c).
 * logdet[f * capacity + slot], f = rgb, depth, obj. slot_of[n] must be filled with -1
 * and n_slots with 0 before the first training view (ngs_hessian_reset). */
typedef struct {
  int32_t k;
  int32_t capacity;
  int32_t* slot_of;    /* [n] */
  int32_t* n_slots;    /* [1] */
  int32_t* gid_of;     /* [capacity] */
  double* h_rgb;
  double* h_d;
  double* h_o;
  double* logdet;      /* [3][capacity] */
  double* trinv;       /* [3][capacity] trace(H_T,g^-1), filled by ngs_hessian_finalize when
                          not NULL; needed by the trace criterion */
} ngs_hessian;

/* Per-view statistics the kernels add into (device, int64 [NGS_STATS_LEN], caller-zeroed):
 * [0] views, [1] pairs M, [2] Gaussians with a nonzero weight that contribute to at
 *     least one pixel U,
 * [3] contributing (pixel, Gaussian) pairs P, [4] walked (tile, entry) pairs, both over
 *     the tiles the information walk visits (with a target object only the tiles that the
 *     rect of a weighted Gaussian reaches; the others add nothing to any statistic),
 * [5] views whose slot workspace overflowed,
 * [6] entries the back-to-front walk stages (per visited tile, from its last contributor
 *     to its first weighted contributor),
 * [7] contributing (pixel, Gaussian) pairs of the back-to-front walk (each updates the
 *     pixel's colour, depth and object suffixes),
 * [8] per-pixel records of weighted contributing pairs (each enters the 94 + 6k products of
 *     the Gaussian's statistics),
 * [9] contributing (tile, Gaussian) pairs F (a Gaussian composited at some pixel of the tile),
 *     over the tiles the information walk visits,
 * [10]-[13] shader-clock cycles (s_memtime) of the back-to-front walk's wavefronts, summed
 *     over them: waiting at the per-batch workgroup barrier, staging a batch of entries into
 *     LDS, walking it, and (a part of the walking) forming and reducing the records of
 *     weighted contributors. A profile of where the walk spends its time, not a count. */
#define NGS_STATS_LEN 14

/* Workspace sizing. op: 0 = ngs_bin_sort, 1 = ngs_info_gain, 2 = ngs_score_batch (and
 * ngs_training_setup, ngs_score_graph_create), 3 = ngs_render_backward,
 * 4 = ngs_sur_render_features (ngs_surrogate.h), 5 = ngs_count_pairs.
 * dims: n, k, width, height, pair capacity, slot capacity, and (ngs_score_batch only)
 * the number of views kept in flight at once, each with its own buffer set (<= 0: 8;
 * at most 64; at most 32 for op 4, where it is the views per grouped render). All host. */
typedef struct {
  int64_t n, k, width, height, max_pairs, max_slots, views_in_flight;
} ngs_dims;

/* ---------------------------------------------------------------------------------
 * Context and helpers
 * --------------------------------------------------------------------------------- */
ngs_status ngs_create(int device, ngs_ctx** out);
ngs_status ngs_destroy(ngs_ctx* ctx);
const char* ngs_status_string(ngs_status s);
int32_t ngs_version(void);
/* Last hipError_t seen by this context (0 if none). */
int32_t ngs_last_hip_error(const ngs_ctx* ctx);
ngs_status ngs_workspace_size(int32_t op, const ngs_dims* dims, size_t* bytes);

/* Per-scene precompute: p = softmax(o) (Sec. III-A.1), sigma, kappa, the confidence
 * c_g of Eq. 7 (target_id < 0) or Eq. 12 (target_id >= 0), labels, and (when cov3 is not
 * NULL) each Gaussian's 3D covariance in FP64. */
ngs_status ngs_prepare_scene(ngs_ctx* ctx, ngs_scene* scene, const ngs_ig_params* ig, void* stream);

/* Projection of every Gaussian for one camera (host struct), following the 3DGS pipeline
 * (Sec. IV-A.2): X = R mu + t, cull Z <= z_near, 2D mean, EWA covariance
 * J R Sigma3 R^T J^T + eps2d I, conic, radius ceil(3 sqrt(lambda_max)), tile rect. The
 * depth key, 2D mean, covariance, radius and rect are evaluated in FP64 in a fixed order
 * without contraction, so keys and rects are reproducible bit for bit. */
ngs_status ngs_project(ngs_ctx* ctx, const ngs_scene* scene, const ngs_camera* cam,
                       const ngs_raster_params* rp, ngs_projected* out, void* stream);

/* Tile binning and sorting of the tile-based rasterizer of the 3DGS pipeline the paper
 * builds on (Sec. IV-A.2; Sec. III-B.1 modifies that rasterizer): every (tile, Gaussian)
 * pair of the rects sorted by (tile, float32 depth bits, gid), and per-tile [start, end)
 * ranges. Radix sort:
 * depth digits over the visible Gaussians, then a stable pass on tile digits over the
 * emitted pairs. Syncs (reads M). If M > capacity returns NGS_CAPACITY with M in
 * *n_pairs. ws: ngs_workspace_size(0, ...) bytes. */
ngs_status ngs_bin_sort(ngs_ctx* ctx, const ngs_scene* scene, const ngs_projected* proj,
                        const ngs_camera* cam, const ngs_raster_params* rp, ngs_tile_lists* out,
                        void* ws, size_t ws_bytes, void* stream);

/* Capacity pre-pass of a scoring batch (run before ngs_score_batch or before capturing
 * ngs_score_graph_create, whose buffers are sized once): projects every candidate of the
 * host camera array (as ngs_project) and writes its number of (tile, Gaussian) pairs of the
 * tile-based rasterizer (Sec. IV-A.2), pairs[v] (device int64 [n_views]), so that
 * dims.max_pairs can be set to max_v pairs[v]. ws: ngs_workspace_size(5, dims) bytes (one
 * view's projection). Stream-ordered, no host synchronisation. */
ngs_status ngs_count_pairs(ngs_ctx* ctx, const ngs_scene* scene, const ngs_camera* cams, int32_t n_views,
                           const ngs_raster_params* rp, int64_t* pairs, void* ws, size_t ws_bytes, void* stream);

/* Front-to-back compositing per 16x16 tile (Eq. 1-2): colour, depth, object vector O,
 * final transmittance, argmax id, mean confidence, contributor count. */
ngs_status ngs_render(ngs_ctx* ctx, const ngs_scene* scene, const ngs_projected* proj,
                      const ngs_tile_lists* lists, const ngs_camera* cam,
                      const ngs_raster_params* rp, ngs_image* out, void* stream);

/* Information of one view (Eq. 6, block diagonal per Gaussian, Sec. III-B.1) with the
 * per-output parameter subsets of Sec. III-B.3 (rgb: 14, depth: 11, object: 11 + k).
 * SCORE mode: ig_out[3] (device, FP64) = IG_f(T, c) = sum_g logdet(H_T,g + c_g A_g) -
 * logdet(H_T,g) (Eq. 5, 6, 9), or with ig->criterion = 1 the trace reduction R_f (see
 * ngs_ig_params; h->trinv then required); h may be NULL (H_T = lambda I). ACCUMULATE mode: adds
 * w_g A_g into h (w_g = c_g, or 1 when conf_on_train = 0); call ngs_hessian_finalize
 * after the last training view. stats (device int64 [NGS_STATS_LEN]) may be NULL.
 * ws: ngs_workspace_size(1, ...) bytes; its slot capacity (max_slots) must cover every
 * Gaussian with c_g > 0 that contributes to a pixel of the view, else NGS_CAPACITY. */
ngs_status ngs_info_gain(ngs_ctx* ctx, const ngs_scene* scene, const ngs_projected* proj,
                         const ngs_tile_lists* lists, const ngs_camera* cam,
                         const ngs_raster_params* rp, const ngs_ig_params* ig, ngs_hessian* h,
                         double* ig_out, int64_t* stats, void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): ngs_info_gain with the same arguments and results,
 * except that its workspace is a fixed array of NGS_STATIC_SCRATCH_BYTES in device memory that
 * the library holds for the rest of the process, one copy per GPU (set up by ngs_create). No
 * allocation or free happens in the call. The array must hold the per-Gaussian and per-pixel
 * tables (about 5 n + 8.5M bytes) and at least one statistics slot, else NGS_WORKSPACE_TOO_SMALL;
 * the slots it holds (about 47k at n = 1M and k = 64) must cover every weighted Gaussian that
 * contributes to a pixel of the view, else NGS_CAPACITY. Every call on one GPU uses the same array: calls that overlap on one GPU
 * (other streams, other contexts, other host threads) race and give undefined results; calls
 * in sequence are independent (each call clears what it reads before use). Syncs like
 * ngs_info_gain. */
#define NGS_STATIC_SCRATCH_BYTES (128u << 20)
ngs_status ngs_info_gain_static(ngs_ctx* ctx, const ngs_scene* scene, const ngs_projected* proj,
                                const ngs_tile_lists* lists, const ngs_camera* cam,
                                const ngs_raster_params* rp, const ngs_ig_params* ig, ngs_hessian* h,
                                double* ig_out, int64_t* stats, void* stream);

/* Clears a training store (slot_of = -1, n_slots = 0). */
ngs_status ngs_hessian_reset(ngs_ctx* ctx, ngs_hessian* h, int32_t n, void* stream);
/* Computes logdet (and trace of the inverse, when h->trinv is given) of every stored
 * block after the last ACCUMULATE view. Syncs; fails
 * with NGS_CAPACITY (needed slots in *n_slots) if a training view overflowed. */
ngs_status ngs_hessian_finalize(ngs_ctx* ctx, ngs_hessian* h, void* stream);

/* Scores n_views candidates (host camera array): per view projection, binning,
 * information gain (SCORE mode), then Eq. 10 normalisation with normalisers[3] (host,
 * the mean training-view gains), Eq. 11 combination and argmax (Eq. 5, lowest index on
 * ties). scores [n_views][4] device FP32: normalised rgb, depth, object, combined.
 * best: device int32. ig_raw [n_views][3] device FP64 receives the raw gains IG_f.
 * stats (device int64 [NGS_STATS_LEN], may be NULL) accumulates (stats[1]: pairs of all
 * views); on return stats[0] = n_views. Returns NGS_DEGENERATE if an enabled normaliser is
 * not positive, NGS_CAPACITY if a view overflows dims->max_pairs or dims->max_slots. ws:
 * ngs_workspace_size(2, dims) bytes, carved by the same dims (host); syncs once per batch.
 * The views run in groups of up to 16 consecutive views, one launch per kernel and group,
 * with ngs_tuning.groups_in_flight groups (default 2) in flight on streams of the context
 * (created on first use, non-blocking, default priority) that wait for the work already
 * queued on `stream` and that `stream` waits for before the combination; each group in
 * flight owns dims->views_in_flight / groups_in_flight consecutive buffer sets and reuses
 * them in stream order. Calls on one context must not overlap. */
ngs_status ngs_score_batch(ngs_ctx* ctx, const ngs_scene* scene, ngs_hessian* h,
                           const double* normalisers, const ngs_camera* cams, int32_t n_views,
                           const ngs_raster_params* rp, const ngs_ig_params* ig, float* scores,
                           int32_t* best, double* ig_raw, int64_t* stats, const ngs_dims* dims,
                           void* ws, size_t ws_bytes, void* stream);

/* Training information and Eq. 10 normalisers of the initial views T (Sec. III-B, Eq. 9-10),
 * in one call: resets the store h, adds c_g A_t,g of every training view t (ACCUMULATE, so
 * H_T = lambda I + sum_t c_g A_t,g), computes the stored blocks' log-dets (and traces of
 * their inverses when h->trinv is given), scores every training view against the finished
 * H_T, and writes (all device FP64, caller-owned):
 *   ig_train [n_train][3]  raw gains IG_f(T, t) (criterion 1: trace reductions R_f);
 *   normalisers [3]        n_f = mean over t of IG_f(T, t) (Eq. 10); criterion 1: the mean
 *                          of the set-function gains R / (S (S - R));
 *   trace_total [3]        (may be NULL) S_f = sum over all n Gaussians of trace(H_T,g^-1),
 *                          Gaussians without a stored block counting l_f / lambda (criterion 1;
 *                          0 otherwise): the value ngs_ig_params.trace_total must carry when
 *                          the candidates are scored.
 * train: host array of n_train cameras. ig: mode is ignored. ws / dims: as for
 * ngs_score_batch (ngs_workspace_size(2, dims) bytes; the training views run one after
 * another on its first buffer set). Syncs. Returns NGS_CAPACITY if a training view exceeds
 * dims->max_pairs or dims->max_slots or the store exceeds h->capacity (needed slots in
 * *h->n_slots), NGS_DEGENERATE if an enabled normaliser is not positive (the outputs are
 * written all the same). */
ngs_status ngs_training_setup(ngs_ctx* ctx, const ngs_scene* scene, ngs_hessian* h, const ngs_camera* train,
                              int32_t n_train, const ngs_raster_params* rp, const ngs_ig_params* ig,
                              double* normalisers, double* trace_total, double* ig_train, const ngs_dims* dims,
                              void* ws, size_t ws_bytes, void* stream);

/* Launch shapes of a context (all calls on it that follow use them; zero fields = defaults).
 * ig_lanes_per_pixel: lanes of the information-gain tile kernel per pixel, 1, 2 or 4: the
 * object channels of a pixel are split over that many lanes, the workgroup has 256 times as
 * many lanes, and a reduction round stages 16 packed rows per wavefront in LDS (8 with 4
 * lanes). Allowed: k <= 8: 1, 2; k <= 32: 1, 2, 4; k <= 64: 1, 2. Default: 1 for k <= 8,
 * else 2. A value not allowed for the scene's k makes ngs_info_gain, ngs_score_batch and
 * ngs_score_graph_create return NGS_INVALID_ARG. Results agree across shapes to rounding.
 * ig_waves_per_simd: 0 (default) or 4: with two lanes per pixel and k > 16, the back pass of
 * the information walk is compiled for four waves per SIMD (two workgroups per CU, a few
 * registers spilled) instead of one workgroup per CU; any other combination makes the calls
 * above return NGS_INVALID_ARG.
 * bin_chunk: least entries per chunk of the second binning level (ngs_bin_sort,
 * ngs_score_batch, ngs_training_setup; 0 = 512, else a power of two in [256, 8192]): longer chunks leave fewer
 * partly written lines in the tile lists, shorter ones spread the scatter over more
 * workgroups. Results do not depend on it.
 * groups_in_flight: ngs_score_batch and ngs_score_graph_create run the views in groups, one
 * launch per kernel and group, with this many groups in flight on context streams (0 = 2,
 * else 1 to 4); a group has views_in_flight / groups_in_flight views (at most 16). Results do
 * not depend on it.
 * The autotuner of the Python package picks these and views_in_flight by timing. */
typedef struct {
  int32_t ig_lanes_per_pixel;
  int32_t ig_waves_per_simd;
  int32_t bin_chunk;
  int32_t groups_in_flight;
} ngs_tuning;
ngs_status ngs_set_tuning(ngs_ctx* ctx, const ngs_tuning* tuning);
ngs_status ngs_get_tuning(const ngs_ctx* ctx, ngs_tuning* tuning);

/* The same batch captured once into a HIP graph and replayed with one launch per batch.
 * ngs_score_graph_create records everything ngs_score_batch enqueues for these arguments
 * (per view on the context's streams: projection, binning, information gain, finalisation;
 * then the combination and argmax) into one graph, instantiates it and returns it in *out;
 * nothing runs. ngs_score_graph_launch replays it on `stream` with a single hipGraphLaunch.
 * Bound by value at capture: the cameras, n_views, rp, ig and dims. Bound by address: the
 * scene arrays, the store h, the workspace and every output, whose contents may change
 * between replays (a refined scene, a grown training store) but not their addresses or
 * sizes. Differences from ngs_score_batch: normalisers is DEVICE memory (FP64 [3]) read at
 * every replay, so the caller can update it between replays; it is not checked, enabled
 * outputs need positive values. overflow (device int32 [1]) is set to 1 by a replay in which
 * some view exceeded dims->max_pairs or dims->max_slots (that view's gains are then not
 * valid) and to 0 otherwise; stats, when given, only accumulates (stats[0] is not written).
 * The graph contains kernel nodes and event dependencies only (no memset or memcpy nodes),
 * no host synchronisation. Replays, and other calls that use the same workspace or context,
 * must not overlap. ngs_score_graph_destroy frees the graph, not the buffers. */
typedef struct ngs_score_graph ngs_score_graph;
ngs_status ngs_score_graph_create(ngs_ctx* ctx, const ngs_scene* scene, ngs_hessian* h, const double* normalisers,
                                  const ngs_camera* cams, int32_t n_views, const ngs_raster_params* rp,
                                  const ngs_ig_params* ig, float* scores, int32_t* best, double* ig_raw,
                                  int64_t* stats, int32_t* overflow, const ngs_dims* dims, void* ws, size_t ws_bytes,
                                  ngs_score_graph** out);
ngs_status ngs_score_graph_launch(ngs_score_graph* graph, void* stream);
ngs_status ngs_score_graph_destroy(ngs_score_graph* graph);

/* Optional kernel timing: while enabled, every kernel the library launches is bracketed
 * by two hipEvents recorded on its launch stream. ngs_profile_read synchronises the
 * recorded events and returns the total milliseconds and launch count of kernel class id
 * (0 <= id < ngs_profile_kernels()); ngs_profile_kernel_name names the class. Enabling
 * (or disabling) clears the totals. The profile is process-wide. */
ngs_status ngs_profile_enable(ngs_ctx* ctx, int32_t on);
/* Like ngs_profile_enable(ctx, 1), but only launches of kernel class id are bracketed, so
 * that timing one kernel adds no events around the others. NGS_INVALID_ARG for an id out of
 * range. ngs_profile_enable(ctx, 0) turns it off. */
ngs_status ngs_profile_enable_class(ngs_ctx* ctx, int32_t id);
int32_t ngs_profile_kernels(void);
const char* ngs_profile_kernel_name(int32_t id);
ngs_status ngs_profile_read(ngs_ctx* ctx, int32_t id, double* total_ms, int64_t* launches);

/* Loss gradients w.r.t. the rendered images (device FP32, layouts as ngs_image): rgb
 * [3][H][W], depth [H][W], obj [k][H][W] (w.r.t. O of Eq. 2, or O' of Eq. 1 when
 * obj_eq2 = 0). A NULL plane counts as zero. */
typedef struct {
  const float* rgb;
  const float* depth;
  const float* obj;
} ngs_image_grad;

/* Gradients w.r.t. the scene parameters (device FP32, planes laid out as in ngs_scene:
 * mean [3][n], log_scale [3][n], rot [4][n] raw quaternion, opacity_logit [n], rgb [3][n],
 * obj_logit [k][n]); every entry is written. */
typedef struct {
  float* mean;
  float* log_scale;
  float* rot;
  float* opacity_logit;
  float* rgb;
  float* obj_logit;
} ngs_scene_grad;

/* Backward rasterizer (scene refinement, Sec. III-A.2; compositing of Eq. 1-2): given dL/d
 * of the rendered colour, depth and object images of one view, writes dL/d of every
 * Gaussian parameter. The scene must be prepared (ngs_prepare_scene); proj and lists are
 * the view's ngs_project / ngs_bin_sort outputs. ws: ngs_workspace_size(3, ...) bytes
 * (n x (16 + k) FP32 screen-space gradients). Stream-ordered, no host synchronisation. */
ngs_status ngs_render_backward(ngs_ctx* ctx, const ngs_scene* scene, const ngs_projected* proj,
                               const ngs_tile_lists* lists, const ngs_camera* cam,
                               const ngs_raster_params* rp, int32_t obj_eq2,
                               const ngs_image_grad* grad_image, ngs_scene_grad* grad_scene,
                               void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* NGS_H */
