// capi.hip -- the extern "C" boundary of libngs (declared in include/ngs.h): argument
// validation, workspace carving, stream ordering and status codes. No C++ exception and
// no HIP error code crosses the boundary; every failure maps to an ngs_status.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "common.hpp"

struct ngs_ctx {
  int device = 0;
  int32_t last_hip = 0;
  int64_t* pinned = nullptr;  // host-pinned scratch for reading device counters
  void* scratch = nullptr;    // this device's copy of the static scratch array (device address)
  int32_t* dev_small = nullptr;  // 256 bytes of device memory for internal results (ngs_sur_pick)
  // Non-blocking streams (default priority) on which ngs_score_batch keeps several views in
  // flight, and the events that fork them from and join them to the caller's stream.
  std::vector<hipStream_t> lanes;
  std::vector<hipEvent_t> lane_done;
  hipEvent_t fork = nullptr;
  // ngs_sur_render_features: the two halves of its double-buffered view groups are free again
  hipEvent_t half_done[2] = {nullptr, nullptr};
  ngs_tuning tuning{};  // launch shapes (ngs_set_tuning); zero = defaults
};

// Workspace of ngs_info_gain_static: a fixed array in device memory, one copy per GPU the
// library runs on, held until the process ends. In host code `scratch` is only a stand-in
// for the symbol; its device address is taken once per device with hipGetSymbolAddress (at
// ngs_create, with the device current) and only that address is handed to kernels.
static __device__ __align__(256) unsigned char scratch[NGS_STATIC_SCRATCH_BYTES];

namespace {

using namespace ngs;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (which must be `device`), taken once.
hipError_t static_scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_addr[device] = ptr;
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

constexpr size_t kAlign = 256;
inline size_t al(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

#define NGS_TRY_HIP(ctx, expr)                         \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) {                            \
      if (ctx) (ctx)->last_hip = (int32_t)e_;          \
      return NGS_HIP_ERROR;                            \
    }                                                  \
  } while (0)

ngs_status check_scene(const ngs_scene* s, bool need_derived) {
  if (!s || s->n < 0 || s->k <= 0) return NGS_INVALID_ARG;
  if (s->k > NGS_MAX_K) return NGS_UNSUPPORTED;
  if (s->n == 0) return NGS_OK;
  if (!s->mean || !s->log_scale || !s->rot || !s->opacity_logit || !s->rgb || !s->obj_logit) return NGS_INVALID_ARG;
  if (need_derived && (!s->prob || !s->opacity || !s->kappa || !s->conf || !s->label)) return NGS_INVALID_ARG;
  return NGS_OK;
}

ngs_status check_cam(const ngs_camera* c, const ngs_raster_params* rp) {
  if (!c || !rp) return NGS_INVALID_ARG;
  if (rp->tile != kTile) return NGS_UNSUPPORTED;
  if (c->width <= 0 || c->height <= 0) return NGS_INVALID_ARG;
  if (!(c->fx > 0.f) || !(c->fy > 0.f) || !std::isfinite(c->cx) || !std::isfinite(c->cy)) return NGS_INVALID_ARG;
  for (int i = 0; i < 9; ++i) if (!std::isfinite(c->R[i])) return NGS_INVALID_ARG;
  for (int i = 0; i < 3; ++i) if (!std::isfinite(c->t[i])) return NGS_INVALID_ARG;
  const int64_t tiles = (int64_t)((c->width + kTile - 1) / kTile) * ((c->height + kTile - 1) / kTile);
  if (tiles > NGS_MAX_TILES) return NGS_UNSUPPORTED;
  if (!(rp->alpha_max > 0.f && rp->alpha_max < 1.f) || !(rp->t_min > 0.f) || !(rp->eps2d >= 0.f)) return NGS_INVALID_ARG;
  return NGS_OK;
}

ngs_status check_proj(const ngs_projected* p) {
  if (!p || !p->mean2d || !p->conic || !p->depth || !p->zkey || !p->rect || !p->count) return NGS_INVALID_ARG;
  return NGS_OK;
}

ngs_status check_lists(const ngs_tile_lists* l) {
  if (!l || !l->gids || !l->ranges || !l->n_pairs || l->capacity < 0) return NGS_INVALID_ARG;
  return NGS_OK;
}

ngs_status check_ig(const ngs_ig_params* ig) {
  if (!ig) return NGS_INVALID_ARG;
  if (!(ig->lambda_prior > 0.f) || ig->outputs == 0u || (ig->outputs & ~7u)) return NGS_INVALID_ARG;
  if (ig->mode != NGS_MODE_SCORE && ig->mode != NGS_MODE_ACCUMULATE) return NGS_INVALID_ARG;
  if (ig->criterion != 0 && ig->criterion != 1) return NGS_INVALID_ARG;
  return NGS_OK;
}

// IG workspace: [256 B header: sticky overflow flag][IgWs regions]
constexpr size_t kIgHeader = 256;

int64_t ig_slots_for(size_t ws_bytes, int64_t n, int64_t k) {
  if (ws_bytes < kIgHeader) return 0;
  const size_t per = (size_t)ig_stat_stride(k) * 4 + 4 + 7 * kNGeo * 8;
  const size_t fixed = ig_ws_fixed_bytes(n) + 4 * kAlign;
  if (ws_bytes < kIgHeader + fixed) return 0;
  int64_t s = (int64_t)((ws_bytes - kIgHeader - fixed) / per);
  while (s > 0 && kIgHeader + ig_ws_bytes(n, k, s) > ws_bytes) --s;
  return s;
}

ngs_status ig_prepare(ngs_ctx* ctx, void* ws, size_t ws_bytes, int64_t n, int64_t k, hipStream_t st, IgWs* w,
                      int32_t** sticky) {
  const int64_t slots = ig_slots_for(ws_bytes, n, k);
  if (slots < 1) return NGS_WORKSPACE_TOO_SMALL;
  *sticky = static_cast<int32_t*>(ws);
  *w = ig_ws_carve(static_cast<char*>(ws) + kIgHeader, n, k, slots);
  NGS_TRY_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t*>(*sticky), 0u, kIgHeader / 4, st));
  NGS_TRY_HIP(ctx, launch_ig_reset_slots(*w, n, st));
  return NGS_OK;
}

ngs_status read_i64(ngs_ctx* ctx, const void* dev, size_t bytes, hipStream_t st, int64_t* out) {
  *ctx->pinned = 0;
  NGS_TRY_HIP(ctx, hipMemcpyAsync(ctx->pinned, dev, bytes, hipMemcpyDeviceToHost, st));
  NGS_TRY_HIP(ctx, hipStreamSynchronize(st));
  if (bytes == 4) {
    int32_t v;
    std::memcpy(&v, ctx->pinned, 4);
    *out = v;
  } else {
    *out = *ctx->pinned;
  }
  return NGS_OK;
}

// Score-batch workspace: projected arrays, lists, binning workspace, IG workspace.
struct BatchWs {
  ngs_projected proj;
  ngs_tile_lists lists;
  void* bin;
  size_t bin_bytes;
  void* ig;
  size_t ig_bytes;
};

size_t batch_fixed_bytes(int64_t n, int64_t max_pairs) {
  const size_t nn = (size_t)std::max<int64_t>(n, 1), mp = (size_t)std::max<int64_t>(max_pairs, 1);
  return al(nn * 8) + al(nn * 12) + al(nn * 4) + al(nn * 4) + al(nn * 8) + al(nn * 4) + al(nn * 32) + al(mp * 4) +
         al(2 * NGS_MAX_TILES * 4) + al(8) + al(bin_ws_bytes(n, max_pairs));
}

// One view's projection arrays (ngs_count_pairs).
size_t proj_set_bytes(int64_t n) {
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  return al(nn * 8) + al(nn * 12) + al(nn * 4) + al(nn * 4) + al(nn * 8) + al(nn * 4);
}

ngs_projected proj_carve(void* ws, int64_t n) {
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t b) { char* r = p; p += al(b); return r; };
  ngs_projected pr;
  pr.mean2d = (float*)take(nn * 8);
  pr.conic = (float*)take(nn * 12);
  pr.depth = (float*)take(nn * 4);
  pr.zkey = (uint32_t*)take(nn * 4);
  pr.rect = (int16_t*)take(nn * 8);
  pr.count = (uint32_t*)take(nn * 4);
  pr.splat = nullptr;  // the pre-pass only counts pairs
  return pr;
}

constexpr int kDefaultInFlight = 8;
constexpr int kMaxInFlight = 64;
constexpr int kMaxGroupsInFlight = 4;  // context streams a scoring batch uses
constexpr int kMaxFeatureGroup = 32;  // views per grouped render launch of the feature maps

int views_in_flight(const ngs_dims* d, int cap = kMaxInFlight) {
  return d->views_in_flight <= 0 ? kDefaultInFlight : (int)std::min<int64_t>(d->views_in_flight, cap);
}

// Creates the context's in-flight streams and events up to `want`.
ngs_status ensure_lanes(ngs_ctx* ctx, int want) {
  if (!ctx->fork) NGS_TRY_HIP(ctx, hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
  for (hipEvent_t& e : ctx->half_done)
    if (!e) NGS_TRY_HIP(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  while ((int)ctx->lanes.size() < want) {
    hipStream_t s = nullptr;
    NGS_TRY_HIP(ctx, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    hipEvent_t e = nullptr;
    hipError_t err = hipEventCreateWithFlags(&e, hipEventDisableTiming);
    if (err != hipSuccess) {
      (void)hipStreamDestroy(s);
      ctx->last_hip = (int32_t)err;
      return NGS_HIP_ERROR;
    }
    ctx->lanes.push_back(s);
    ctx->lane_done.push_back(e);
  }
  return NGS_OK;
}

// One 80 x 60 render (rgb, depth, t_final, mean_conf, argmax id) for the feature maps.
size_t feat_img_bytes() {
  const size_t hw = (size_t)NGS_SUR_IN_W * NGS_SUR_IN_H;
  return 7 * al(hw * 4);
}

ngs_image feat_img_carve(char* p) {
  const size_t hw = (size_t)NGS_SUR_IN_W * NGS_SUR_IN_H;
  ngs_image im{};
  im.rgb = (float*)p; p += 3 * al(hw * 4);
  im.depth = (float*)p; p += al(hw * 4);
  im.t_final = (float*)p; p += al(hw * 4);
  im.mean_conf = (float*)p; p += al(hw * 4);
  im.argmax_id = (int32_t*)p;
  im.obj = nullptr;
  im.n_contrib = nullptr;
  return im;
}

// The projection outputs that the information walks read: the 2D means and conics are in the
// splat records, so their separate arrays are not written.
ngs_projected walk_only(ngs_projected p) {
  p.mean2d = nullptr;
  p.conic = nullptr;
  return p;
}

BatchWs batch_carve(void* ws, size_t ws_bytes, int64_t n, int64_t max_pairs) {
  const size_t nn = (size_t)std::max<int64_t>(n, 1), mp = (size_t)std::max<int64_t>(max_pairs, 1);
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t b) { char* r = p; p += al(b); return r; };
  BatchWs b;
  b.proj.mean2d = (float*)take(nn * 8);
  b.proj.conic = (float*)take(nn * 12);
  b.proj.depth = (float*)take(nn * 4);
  b.proj.zkey = (uint32_t*)take(nn * 4);
  b.proj.rect = (int16_t*)take(nn * 8);
  b.proj.count = (uint32_t*)take(nn * 4);
  b.proj.splat = (float*)take(nn * 32);
  b.lists.gids = (uint32_t*)take(mp * 4);
  b.lists.ranges = (uint32_t*)take(2 * NGS_MAX_TILES * 4);
  b.lists.n_pairs = (int64_t*)take(8);
  b.lists.keys = nullptr;
  b.lists.capacity = max_pairs;
  b.bin_bytes = al(bin_ws_bytes(n, max_pairs));
  b.bin = take(b.bin_bytes);
  b.ig = p;
  const size_t used = (size_t)(p - static_cast<char*>(ws));
  b.ig_bytes = ws_bytes > used ? ws_bytes - used : 0;
  return b;
}

}  // namespace

extern "C" {

ngs_status ngs_create(int device, ngs_ctx** out) {
  if (!out) return NGS_INVALID_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return NGS_INVALID_ARG;
  ngs_ctx* c = new (std::nothrow) ngs_ctx();
  if (!c) return NGS_HIP_ERROR;
  c->device = device;
  hipError_t e = hipSetDevice(device);
  if (e == hipSuccess) e = hipHostMalloc((void**)&c->pinned, 64, hipHostMallocDefault);
  if (e == hipSuccess) e = static_scratch_address(device, &c->scratch);
  if (e == hipSuccess) e = hipMalloc((void**)&c->dev_small, 256);
  if (e != hipSuccess) {
    if (c->pinned) (void)hipHostFree(c->pinned);
    delete c;
    return NGS_HIP_ERROR;
  }
  *out = c;
  return NGS_OK;
}

ngs_status ngs_destroy(ngs_ctx* ctx) {
  if (!ctx) return NGS_INVALID_ARG;
  (void)hipSetDevice(ctx->device);
  for (hipStream_t s : ctx->lanes) (void)hipStreamDestroy(s);
  for (hipEvent_t e : ctx->lane_done) (void)hipEventDestroy(e);
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  for (hipEvent_t e : ctx->half_done)
    if (e) (void)hipEventDestroy(e);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->dev_small) (void)hipFree(ctx->dev_small);
  delete ctx;
  return NGS_OK;
}

const char* ngs_status_string(ngs_status s) {
  switch (s) {
    case NGS_OK: return "ok";
    case NGS_INVALID_ARG: return "invalid argument";
    case NGS_CAPACITY: return "output capacity too small";
    case NGS_WORKSPACE_TOO_SMALL: return "workspace too small";
    case NGS_HIP_ERROR: return "HIP runtime error";
    case NGS_DEGENERATE: return "degenerate normaliser";
    case NGS_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
  }
}

int32_t ngs_version(void) { return 1; }

int32_t ngs_last_hip_error(const ngs_ctx* ctx) { return ctx ? ctx->last_hip : 0; }

ngs_status ngs_workspace_size(int32_t op, const ngs_dims* d, size_t* bytes) {
  if (!d || !bytes || d->n < 0 || d->k <= 0 || d->max_pairs < 0 || d->max_slots < 0) return NGS_INVALID_ARG;
  if (d->k > NGS_MAX_K) return NGS_UNSUPPORTED;
  const size_t igb = kIgHeader + ig_ws_bytes(d->n, d->k, std::max<int64_t>(d->max_slots, 1));
  switch (op) {
    case 0: *bytes = bin_ws_bytes(d->n, d->max_pairs); return NGS_OK;
    case 1: *bytes = igb; return NGS_OK;
    case 2: *bytes = (size_t)views_in_flight(d) * al(batch_fixed_bytes(d->n, d->max_pairs) + igb); return NGS_OK;
    case 3: *bytes = bwd_ws_bytes(d->n, d->k); return NGS_OK;
    case 4:
      *bytes = kIgHeader + 2 * (size_t)views_in_flight(d, kMaxFeatureGroup) *
                               al(batch_fixed_bytes(d->n, d->max_pairs) + feat_img_bytes());
      return NGS_OK;
    case 5: *bytes = proj_set_bytes(d->n); return NGS_OK;
    default: return NGS_INVALID_ARG;
  }
}

ngs_status ngs_prepare_scene(ngs_ctx* ctx, ngs_scene* scene, const ngs_ig_params* ig, void* stream) {
  if (!ctx) return NGS_INVALID_ARG;
  ngs_status s = check_scene(scene, true);
  if (s != NGS_OK) return s;
  if (!ig) return NGS_INVALID_ARG;
  if (ig->target_id >= scene->k) return NGS_INVALID_ARG;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  NGS_TRY_HIP(ctx, launch_prepare_scene(*scene, *ig, (hipStream_t)stream));
  return NGS_OK;
}

ngs_status ngs_project(ngs_ctx* ctx, const ngs_scene* scene, const ngs_camera* cam, const ngs_raster_params* rp,
                       ngs_projected* out, void* stream) {
  if (!ctx) return NGS_INVALID_ARG;
  ngs_status s = check_scene(scene, false);
  if (s == NGS_OK) s = check_cam(cam, rp);
  if (s == NGS_OK) s = check_proj(out);
  if (s != NGS_OK) return s;
  if (out->splat && scene->n > 0 && !scene->opacity) return NGS_INVALID_ARG;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  NGS_TRY_HIP(ctx, launch_project(*scene, single_group(make_devcam(*cam, kTile)), *rp, *out, (hipStream_t)stream));
  return NGS_OK;
}

ngs_status ngs_bin_sort(ngs_ctx* ctx, const ngs_scene* scene, const ngs_projected* proj, const ngs_camera* cam,
                        const ngs_raster_params* rp, ngs_tile_lists* out, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return NGS_INVALID_ARG;
  ngs_status s = check_scene(scene, false);
  if (s == NGS_OK) s = check_cam(cam, rp);
  if (s == NGS_OK) s = check_proj(proj);
  if (s == NGS_OK) s = check_lists(out);
  if (s != NGS_OK) return s;
  if (!ws || ws_bytes < bin_ws_bytes(scene->n, out->capacity)) return NGS_WORKSPACE_TOO_SMALL;
  hipStream_t st = (hipStream_t)stream;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  const Group G1 = single_group(make_devcam(*cam, kTile));
  const BinWs w = bin_ws_carve(ws, scene->n, out->capacity);
  NGS_TRY_HIP(ctx, bin_count_pairs(*proj, scene->n, w, st));
  int64_t m = 0;
  s = read_i64(ctx, w.m_total, 8, st, &m);
  if (s != NGS_OK) return s;
  if (m > out->capacity || m >= (int64_t)UINT32_MAX) {
    NGS_TRY_HIP(ctx, hipMemcpyAsync(out->n_pairs, w.m_total, 8, hipMemcpyDeviceToDevice, st));
    NGS_TRY_HIP(ctx, hipStreamSynchronize(st));
    return m >= (int64_t)UINT32_MAX ? NGS_UNSUPPORTED : NGS_CAPACITY;
  }
  NGS_TRY_HIP(ctx, bin_emit_and_sort(*proj, scene->n, G1, w, *out, nullptr, nullptr, st, nullptr, ctx->tuning.bin_chunk));
  return NGS_OK;
}

ngs_status ngs_count_pairs(ngs_ctx* ctx, const ngs_scene* scene, const ngs_camera* cams, int32_t n_views,
                           const ngs_raster_params* rp, int64_t* pairs, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !cams || n_views < 0 || !pairs) return NGS_INVALID_ARG;
  ngs_status s = check_scene(scene, false);
  if (s != NGS_OK) return s;
  for (int v = 0; v < n_views; ++v) {
    s = check_cam(&cams[v], rp);
    if (s != NGS_OK) return s;
  }
  if (!ws || ws_bytes < proj_set_bytes(scene->n)) return NGS_WORKSPACE_TOO_SMALL;
  hipStream_t st = (hipStream_t)stream;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  const ngs_projected pr = proj_carve(ws, scene->n);
  NGS_TRY_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t*>(pairs), 0u, 2 * (size_t)n_views, st));
  for (int v = 0; v < n_views; ++v) {
    NGS_TRY_HIP(ctx, launch_project(*scene, single_group(make_devcam(cams[v], kTile)), *rp, pr, st));
    NGS_TRY_HIP(ctx, launch_sum_counts(pr, scene->n, pairs + v, st));
  }
  return NGS_OK;
}

ngs_status ngs_render(ngs_ctx* ctx, const ngs_scene* scene, const ngs_projected* proj, const ngs_tile_lists* lists,
                      const ngs_camera* cam, const ngs_raster_params* rp, ngs_image* out, void* stream) {
  if (!ctx) return NGS_INVALID_ARG;
  ngs_status s = check_scene(scene, true);
  if (s == NGS_OK) s = check_cam(cam, rp);
  if (s == NGS_OK) s = check_proj(proj);
  if (s == NGS_OK) s = check_lists(lists);
  if (s != NGS_OK) return s;
  if (!out || !out->rgb || !out->depth || !out->t_final || !out->argmax_id) return NGS_INVALID_ARG;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  NGS_TRY_HIP(ctx, launch_render(*scene, *proj, *lists, make_devcam(*cam, kTile), make_raster(*rp), *out,
                                 (hipStream_t)stream));
  return NGS_OK;
}

ngs_status ngs_hessian_reset(ngs_ctx* ctx, ngs_hessian* h, int32_t n, void* stream) {
  if (!ctx || !h || n < 0 || !h->slot_of || !h->n_slots) return NGS_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  NGS_TRY_HIP(ctx, launch_fill_i32(h->slot_of, -1, (size_t)n, st));
  NGS_TRY_HIP(ctx, hipMemsetAsync(h->n_slots, 0, 4, st));
  return NGS_OK;
}

ngs_status ngs_hessian_finalize(ngs_ctx* ctx, ngs_hessian* h, void* stream) {
  if (!ctx || !h || !h->n_slots || !h->logdet || !h->h_rgb || !h->h_d || !h->h_o || h->capacity < 0) return NGS_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  int64_t used = 0;
  ngs_status s = read_i64(ctx, h->n_slots, 4, st, &used);
  if (s != NGS_OK) return s;
  if (used > h->capacity) return NGS_CAPACITY;
  NGS_TRY_HIP(ctx, launch_hessian_logdet(h, (int32_t)used, 0.f, st));
  return NGS_OK;
}

ngs_status ngs_info_gain(ngs_ctx* ctx, const ngs_scene* scene, const ngs_projected* proj, const ngs_tile_lists* lists,
                         const ngs_camera* cam, const ngs_raster_params* rp, const ngs_ig_params* ig, ngs_hessian* h,
                         double* ig_out, int64_t* stats, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx) return NGS_INVALID_ARG;
  ngs_status s = check_scene(scene, true);
  if (s == NGS_OK) s = check_cam(cam, rp);
  if (s == NGS_OK) s = check_proj(proj);
  if (s == NGS_OK) s = check_lists(lists);
  if (s == NGS_OK) s = check_ig(ig);
  if (s != NGS_OK) return s;
  if (ig->mode == NGS_MODE_ACCUMULATE && (!h || !h->slot_of || !h->n_slots || !h->gid_of || !h->h_rgb || !h->h_d || !h->h_o))
    return NGS_INVALID_ARG;
  if (ig->mode == NGS_MODE_SCORE && !ig_out) return NGS_INVALID_ARG;
  if (!proj->splat && scene->n > 0) return NGS_INVALID_ARG;
  if (h && (h->k != scene->k || (h->capacity > 0 && !h->logdet))) return NGS_INVALID_ARG;
  if (ig->criterion == 1 && ig->mode == NGS_MODE_SCORE && h && h->capacity > 0 && !h->trinv) return NGS_INVALID_ARG;
  if (!ig_lpp_valid(scene->k, ctx->tuning.ig_lanes_per_pixel) ||
      !ig_waves_valid(scene->k, ctx->tuning.ig_lanes_per_pixel, ctx->tuning.ig_waves_per_simd))
    return NGS_INVALID_ARG;
  if (!ws) return NGS_WORKSPACE_TOO_SMALL;
  hipStream_t st = (hipStream_t)stream;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  IgWs w;
  int32_t* sticky = nullptr;
  s = ig_prepare(ctx, ws, ws_bytes, scene->n, scene->k, st, &w, &sticky);
  if (s != NGS_OK) return s;
  if (ig_out) NGS_TRY_HIP(ctx, hipMemsetAsync(ig_out, 0, 3 * sizeof(double), st));
  const Group G1 = single_group(make_devcam(*cam, kTile));
  NGS_TRY_HIP(ctx, launch_ig_tiles(*scene, *proj, *lists, G1, make_raster(*rp), *ig, w, stats, ctx->tuning.ig_lanes_per_pixel,
                                   st, ctx->tuning.ig_waves_per_simd));
  NGS_TRY_HIP(ctx, launch_ig_finalize(*scene, G1, *rp, *ig, w, h, ig_out ? ig_out : nullptr, stats, sticky, st));
  int64_t of = 0;
  s = read_i64(ctx, sticky, 4, st, &of);
  if (s != NGS_OK) return s;
  if (of) {
    NGS_TRY_HIP(ctx, hipMemsetAsync(sticky, 0, 4, st));
    return NGS_CAPACITY;
  }
  return NGS_OK;
}

ngs_status ngs_info_gain_static(ngs_ctx* ctx, const ngs_scene* scene, const ngs_projected* proj,
                                const ngs_tile_lists* lists, const ngs_camera* cam, const ngs_raster_params* rp,
                                const ngs_ig_params* ig, ngs_hessian* h, double* ig_out, int64_t* stats,
                                void* stream) {
  if (!ctx || !ctx->scratch) return NGS_INVALID_ARG;
  if (!scene || scene->n < 0 || scene->k <= 0) return NGS_INVALID_ARG;
  if (scene->k > NGS_MAX_K) return NGS_UNSUPPORTED;
  // the slot statistics of ngs_info_gain must fit the fixed array: at least one slot
  if (ig_slots_for(NGS_STATIC_SCRATCH_BYTES, scene->n, scene->k) < 1) return NGS_WORKSPACE_TOO_SMALL;
  // every call on this device shares the array; ngs_info_gain clears what must start at zero
  return ngs_info_gain(ctx, scene, proj, lists, cam, rp, ig, h, ig_out, stats, ctx->scratch,
                       NGS_STATIC_SCRATCH_BYTES, stream);
}

}  // extern "C"

namespace {

// Checks shared by ngs_score_batch and ngs_score_graph_create.
ngs_status check_batch(const ngs_scene* scene, ngs_hessian* h, const ngs_camera* cams, int32_t n_views,
                       const ngs_raster_params* rp, const ngs_ig_params* ig, const ngs_dims* dims, void* ws,
                       size_t ws_bytes) {
  if (dims->n != scene->n || dims->k != scene->k || dims->max_pairs < 1 || dims->max_slots < 1) return NGS_INVALID_ARG;
  ngs_status s = check_scene(scene, true);
  if (s == NGS_OK) s = check_ig(ig);
  if (s != NGS_OK) return s;
  if (ig->mode != NGS_MODE_SCORE) return NGS_INVALID_ARG;
  if (h && h->k != scene->k) return NGS_INVALID_ARG;
  if (ig->criterion == 1) {
    if (h && h->capacity > 0 && !h->trinv) return NGS_INVALID_ARG;
    for (int f = 0; f < 3; ++f)
      if (((ig->outputs >> f) & 1u) && !(ig->trace_total[f] > 0.0)) return NGS_INVALID_ARG;
  }
  for (int v = 0; v < n_views; ++v) {
    s = check_cam(&cams[v], rp);
    if (s != NGS_OK) return s;
  }
  if (!ws) return NGS_WORKSPACE_TOO_SMALL;
  size_t need = 0;
  s = ngs_workspace_size(2, dims, &need);
  if (s != NGS_OK) return s;
  return ws_bytes < need ? NGS_WORKSPACE_TOO_SMALL : NGS_OK;
}

// Enqueues a whole scoring batch on `st` and the context streams, with no host
// synchronisation and no memset or memcpy nodes, so that it can also be captured into a
// graph. Normalisers come from nf_dev (device) when given, else from nf_host. *sticky_out
// receives the device flag that a list or slot overflow raises.
ngs_status enqueue_score_batch(ngs_ctx* ctx, const ngs_scene* scene, ngs_hessian* h, const double* nf_host,
                               const double* nf_dev, const ngs_camera* cams, int32_t n_views,
                               const ngs_raster_params* rp, const ngs_ig_params* ig, float* scores, int32_t* best,
                               double* ig_raw, int64_t* stats, const ngs_dims* dims, void* ws, hipStream_t st,
                               int32_t** sticky_out) {
  size_t need = 0;
  ngs_status s = ngs_workspace_size(2, dims, &need);
  if (s != NGS_OK) return s;
  const int64_t max_pairs = dims->max_pairs;
  const int lanes = std::max(1, std::min(views_in_flight(dims), n_views));
  // one buffer set per in-flight view; the first set's IG header holds the sticky overflow
  // flag that every set reports into
  const size_t per = need / (size_t)views_in_flight(dims);
  std::vector<BatchWs> sets(lanes);
  std::vector<IgWs> igs(lanes);
  int32_t* sticky = nullptr;
  for (int i = 0; i < lanes; ++i) {
    sets[i] = batch_carve(static_cast<char*>(ws) + (size_t)i * per, per, scene->n, max_pairs);
    int32_t* own = nullptr;
    s = ig_prepare(ctx, sets[i].ig, sets[i].ig_bytes, scene->n, scene->k, st, &igs[i], &own);
    if (s != NGS_OK) return s;
    if (i == 0) sticky = own;
  }
  *sticky_out = sticky;
  NGS_TRY_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t*>(ig_raw), 0u, (size_t)6 * std::max(n_views, 1), st));
  // List overflow is caught on the device (empty ranges, sticky flag) and reported once the
  // batch has run. Views go in groups of gsz consecutive views, one launch per kernel and
  // group (grid.y = view of the group); the buffer sets of a group are consecutive, per bytes
  // apart. nlanes groups are in flight: group q runs on lane q mod nlanes with the sets from
  // (q mod nlanes) * gsz on, which it reuses in stream order.
  const int nlanes = std::max(1, std::min(ctx->tuning.groups_in_flight > 0 ? ctx->tuning.groups_in_flight : 2, lanes));
  const int gsz = std::max(1, std::min(kMaxGroup, lanes / nlanes));
  NGS_TRY_HIP(ctx, hipEventRecord(ctx->fork, st));
  for (int i = 0; i < nlanes; ++i) NGS_TRY_HIP(ctx, hipStreamWaitEvent(ctx->lanes[i], ctx->fork, 0));
  std::vector<DevCam> dcs(n_views);
  for (int v = 0; v < n_views; ++v) dcs[v] = make_devcam(cams[v], kTile);
  for (int v0 = 0, q = 0; v0 < n_views; v0 += gsz, ++q) {
    const int g = std::min(gsz, n_views - v0);
    const int i = (q % nlanes) * gsz;
    hipStream_t ls = ctx->lanes[q % nlanes];
    const BatchWs& b = sets[i];
    const BinWs bw = bin_ws_carve(b.bin, scene->n, max_pairs);
    const Group G = make_group(&dcs[v0], g, per);
    // with a target object the projection also flags the tiles that a weighted Gaussian
    // reaches: only their lists are written, the only ones the information walk reads
    NGS_TRY_HIP(ctx, launch_ig_clear(*ig, igs[i], G, ls));
    NGS_TRY_HIP(ctx, launch_project(*scene, G, *rp, walk_only(b.proj), ls, 1,
                                    const_cast<int32_t*>(ig_tile_flags(*ig, igs[i]))));
    NGS_TRY_HIP(ctx, bin_count_pairs(b.proj, scene->n, bw, ls, g, per));
    NGS_TRY_HIP(ctx, bin_emit_and_sort(b.proj, scene->n, G, bw, b.lists, sticky, stats, ls, ig_tile_flags(*ig, igs[i]),
                                       ctx->tuning.bin_chunk));
    NGS_TRY_HIP(ctx, launch_ig_walk(*scene, b.proj, b.lists, G, make_raster(*rp), *ig, igs[i], stats,
                                    ctx->tuning.ig_lanes_per_pixel, ls, ctx->tuning.ig_waves_per_simd));
    NGS_TRY_HIP(ctx, launch_ig_finalize(*scene, G, *rp, *ig, igs[i], h, ig_raw + 3 * (size_t)v0, stats, sticky, ls));
  }
  for (int i = 0; i < nlanes; ++i) {
    NGS_TRY_HIP(ctx, hipEventRecord(ctx->lane_done[i], ctx->lanes[i]));
    NGS_TRY_HIP(ctx, hipStreamWaitEvent(st, ctx->lane_done[i], 0));
  }
  const double n0 = nf_host ? nf_host[0] : 1.0, n1 = nf_host ? nf_host[1] : 1.0, n2 = nf_host ? nf_host[2] : 1.0;
  NGS_TRY_HIP(ctx, launch_score_combine(ig_raw, n_views, n0, n1, n2, nf_dev, *ig, scores, best, st));
  return NGS_OK;
}

}  // namespace

extern "C" ngs_status ngs_training_setup(ngs_ctx* ctx, const ngs_scene* scene, ngs_hessian* h,
                                         const ngs_camera* train, int32_t n_train, const ngs_raster_params* rp,
                                         const ngs_ig_params* ig, double* normalisers, double* trace_total,
                                         double* ig_train, const ngs_dims* dims, void* ws, size_t ws_bytes,
                                         void* stream) {
  if (!ctx || !scene || !h || !train || n_train < 1 || !rp || !ig || !normalisers || !ig_train || !dims)
    return NGS_INVALID_ARG;
  if (!h->slot_of || !h->n_slots || !h->gid_of || !h->h_rgb || !h->h_d || !h->h_o || !h->logdet || h->capacity < 1)
    return NGS_INVALID_ARG;
  if (ig->criterion == 1 && !h->trinv) return NGS_INVALID_ARG;
  ngs_ig_params acc = *ig, sc = *ig;
  acc.mode = NGS_MODE_ACCUMULATE;
  sc.mode = NGS_MODE_SCORE;
  // check_batch validates the scene, the cameras and the workspace against dims
  ngs_status s = check_batch(scene, h, train, n_train, rp, &sc, dims, ws, ws_bytes);
  if (s == NGS_INVALID_ARG && ig->criterion == 1) {
    // S_f is what this call computes: validate without it
    for (int f = 0; f < 3; ++f) sc.trace_total[f] = 1.0;
    s = check_batch(scene, h, train, n_train, rp, &sc, dims, ws, ws_bytes);
    sc.trace_total[0] = sc.trace_total[1] = sc.trace_total[2] = 0.0;
  }
  if (s != NGS_OK) return s;
  if (!ig_lpp_valid(scene->k, ctx->tuning.ig_lanes_per_pixel) ||
      !ig_waves_valid(scene->k, ctx->tuning.ig_lanes_per_pixel, ctx->tuning.ig_waves_per_simd))
    return NGS_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  size_t need = 0;
  s = ngs_workspace_size(2, dims, &need);
  if (s != NGS_OK) return s;
  // the training views run one after another on buffer set 0
  const size_t per = need / (size_t)views_in_flight(dims);
  const BatchWs b = batch_carve(ws, per, scene->n, dims->max_pairs);
  IgWs w;
  int32_t* sticky = nullptr;
  s = ig_prepare(ctx, b.ig, b.ig_bytes, scene->n, scene->k, st, &w, &sticky);
  if (s != NGS_OK) return s;
  const BinWs bw = bin_ws_carve(b.bin, scene->n, dims->max_pairs);
  const RasterConst rc = make_raster(*rp);
  const int lpp = ctx->tuning.ig_lanes_per_pixel;
  // H_T = lambda I + sum_t c_g A_t,g (Eq. 9 with the prior)
  NGS_TRY_HIP(ctx, launch_fill_i32(h->slot_of, -1, (size_t)scene->n, st));
  NGS_TRY_HIP(ctx, launch_fill_i32(h->n_slots, 0, 1, st));
  NGS_TRY_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t*>(ig_train), 0u, (size_t)6 * n_train, st));
  for (int pass = 0; pass < 2; ++pass) {
    const ngs_ig_params& p = pass == 0 ? acc : sc;
    for (int t = 0; t < n_train; ++t) {
      const Group G1 = single_group(make_devcam(train[t], kTile));
      NGS_TRY_HIP(ctx, launch_project(*scene, G1, *rp, walk_only(b.proj), st, 1));
      NGS_TRY_HIP(ctx, bin_count_pairs(b.proj, scene->n, bw, st));
      NGS_TRY_HIP(ctx, launch_ig_assign(*scene, b.proj, G1, p, w, st));
      NGS_TRY_HIP(ctx, bin_emit_and_sort(b.proj, scene->n, G1, bw, b.lists, sticky, nullptr, st, ig_tile_flags(p, w),
                                         ctx->tuning.bin_chunk));
      NGS_TRY_HIP(ctx, launch_ig_walk(*scene, b.proj, b.lists, G1, rc, p, w, nullptr, lpp, st,
                                      ctx->tuning.ig_waves_per_simd));
      NGS_TRY_HIP(ctx, launch_ig_finalize(*scene, G1, *rp, p, w, h, pass == 0 ? nullptr : ig_train + 3 * (size_t)t,
                                          nullptr, sticky, st));
    }
    if (pass == 0) {
      // a view beyond the pair or slot capacity, or a store beyond its capacity, stops here
      int64_t of = 0, used = 0;
      s = read_i64(ctx, sticky, 4, st, &of);
      if (s == NGS_OK) s = read_i64(ctx, h->n_slots, 4, st, &used);
      if (s != NGS_OK) return s;
      if (of || used > h->capacity) {
        NGS_TRY_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t*>(sticky), 0u, 1, st));
        return NGS_CAPACITY;
      }
      NGS_TRY_HIP(ctx, launch_hessian_logdet(h, (int32_t)used, ig->lambda_prior, st));
    }
  }
  NGS_TRY_HIP(ctx, launch_train_normalisers(*h, scene->n, scene->k, *ig, ig_train, n_train, normalisers, trace_total,
                                            st));
  int64_t of = 0;
  s = read_i64(ctx, sticky, 4, st, &of);
  if (s != NGS_OK) return s;
  if (of) {
    NGS_TRY_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t*>(sticky), 0u, 1, st));
    return NGS_CAPACITY;
  }
  // Eq. 10 needs positive normalisers for the enabled outputs
  NGS_TRY_HIP(ctx, hipMemcpyAsync(ctx->pinned, normalisers, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
  NGS_TRY_HIP(ctx, hipStreamSynchronize(st));
  double nf[3];
  std::memcpy(nf, ctx->pinned, sizeof nf);
  for (int f = 0; f < 3; ++f)
    if (((ig->outputs >> f) & 1u) && !(nf[f] > 0.0)) return NGS_DEGENERATE;
  return NGS_OK;
}

struct ngs_score_graph {
  ngs_ctx* ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

ngs_status ngs_score_batch(ngs_ctx* ctx, const ngs_scene* scene, ngs_hessian* h, const double* normalisers,
                           const ngs_camera* cams, int32_t n_views, const ngs_raster_params* rp,
                           const ngs_ig_params* ig, float* scores, int32_t* best, double* ig_raw, int64_t* stats,
                           const ngs_dims* dims, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !normalisers || !cams || n_views < 0 || !scores || !best || !ig_raw || !dims || !scene || !rp || !ig)
    return NGS_INVALID_ARG;
  ngs_status s = check_batch(scene, h, cams, n_views, rp, ig, dims, ws, ws_bytes);
  if (s != NGS_OK) return s;
  if (!ig_lpp_valid(scene->k, ctx->tuning.ig_lanes_per_pixel) ||
      !ig_waves_valid(scene->k, ctx->tuning.ig_lanes_per_pixel, ctx->tuning.ig_waves_per_simd))
    return NGS_INVALID_ARG;
  for (int f = 0; f < 3; ++f)
    if (((ig->outputs >> f) & 1u) && !(normalisers[f] > 0.0)) return NGS_DEGENERATE;
  hipStream_t st = (hipStream_t)stream;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  s = ensure_lanes(ctx, std::max(1, std::min(kMaxGroupsInFlight, std::min(views_in_flight(dims), n_views))));
  if (s != NGS_OK) return s;
  int32_t* sticky = nullptr;
  s = enqueue_score_batch(ctx, scene, h, normalisers, nullptr, cams, n_views, rp, ig, scores, best, ig_raw, stats,
                          dims, ws, st, &sticky);
  if (s != NGS_OK) return s;
  int64_t of = 0;
  s = read_i64(ctx, sticky, 4, st, &of);
  if (s != NGS_OK) return s;
  if (stats) {
    ctx->pinned[0] = n_views;
    NGS_TRY_HIP(ctx, hipMemcpyAsync(stats, ctx->pinned, 8, hipMemcpyHostToDevice, st));
    NGS_TRY_HIP(ctx, hipStreamSynchronize(st));
  }
  if (of) {
    NGS_TRY_HIP(ctx, hipMemsetAsync(sticky, 0, 4, st));
    return NGS_CAPACITY;
  }
  return NGS_OK;
}

ngs_status ngs_sur_pick(ngs_ctx* ctx, const ngs_scene* scene, ngs_hessian* h, const double* normalisers,
                        const ngs_camera* cams, int32_t n_views, const float* pred, int32_t rescore,
                        const ngs_raster_params* rp, const ngs_ig_params* ig, int32_t* chosen, float* scores,
                        double* ig_raw, int32_t* best, int64_t* stats, const ngs_dims* dims, void* ws,
                        size_t ws_bytes, void* stream) {
  if (!ctx || !cams || n_views < 1 || !pred || rescore < 1 || !chosen || !scores || !ig_raw || !best)
    return NGS_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  // the network's ranking: candidates by descending prediction, lower index first on ties,
  // a prediction that is not a number last
  std::vector<float> p((size_t)n_views);
  NGS_TRY_HIP(ctx, hipMemcpyAsync(p.data(), pred, p.size() * sizeof(float), hipMemcpyDeviceToHost, st));
  NGS_TRY_HIP(ctx, hipStreamSynchronize(st));
  std::vector<int32_t> order((size_t)n_views);
  for (int32_t v = 0; v < n_views; ++v) order[v] = v;
  const int32_t r = std::min(rescore, n_views);
  auto ahead = [&](int32_t a, int32_t b) {
    const bool na = std::isnan(p[a]), nb = std::isnan(p[b]);
    if (na != nb) return nb;
    if (!na && p[a] != p[b]) return p[a] > p[b];
    return a < b;
  };
  std::partial_sort(order.begin(), order.begin() + r, order.end(), ahead);
  std::vector<ngs_camera> sel((size_t)r);
  for (int32_t i = 0; i < r; ++i) {
    chosen[i] = order[i];
    sel[i] = cams[order[i]];
  }
  // the exact information gain judges the network's choice
  ngs_status s = ngs_score_batch(ctx, scene, h, normalisers, sel.data(), r, rp, ig, scores, ctx->dev_small, ig_raw,
                                 stats, dims, ws, ws_bytes, stream);
  if (s != NGS_OK) return s;
  int64_t local = -1;
  s = read_i64(ctx, ctx->dev_small, 4, st, &local);
  if (s != NGS_OK) return s;
  *best = (local >= 0 && local < r) ? chosen[local] : -1;
  return NGS_OK;
}

ngs_status ngs_score_graph_create(ngs_ctx* ctx, const ngs_scene* scene, ngs_hessian* h, const double* normalisers,
                                  const ngs_camera* cams, int32_t n_views, const ngs_raster_params* rp,
                                  const ngs_ig_params* ig, float* scores, int32_t* best, double* ig_raw,
                                  int64_t* stats, int32_t* overflow, const ngs_dims* dims, void* ws, size_t ws_bytes,
                                  ngs_score_graph** out) {
  if (!out) return NGS_INVALID_ARG;
  *out = nullptr;
  if (!ctx || !normalisers || !cams || n_views < 1 || !scores || !best || !ig_raw || !overflow || !dims || !scene ||
      !rp || !ig)
    return NGS_INVALID_ARG;
  ngs_status s = check_batch(scene, h, cams, n_views, rp, ig, dims, ws, ws_bytes);
  if (s != NGS_OK) return s;
  if (!ig_lpp_valid(scene->k, ctx->tuning.ig_lanes_per_pixel) ||
      !ig_waves_valid(scene->k, ctx->tuning.ig_lanes_per_pixel, ctx->tuning.ig_waves_per_simd))
    return NGS_INVALID_ARG;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  s = ensure_lanes(ctx, std::max(1, std::min(kMaxGroupsInFlight, std::min(views_in_flight(dims), n_views))));
  if (s != NGS_OK) return s;
  hipStream_t cs = nullptr;
  NGS_TRY_HIP(ctx, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  const bool prof = prof_suspend();
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    int32_t* sticky = nullptr;
    s = enqueue_score_batch(ctx, scene, h, nullptr, normalisers, cams, n_views, rp, ig, scores, best, ig_raw, stats,
                            dims, ws, cs, &sticky);
    if (s == NGS_OK) {
      e = launch_copy_u32(reinterpret_cast<uint32_t*>(overflow), reinterpret_cast<const uint32_t*>(sticky), 1, cs);
      if (e != hipSuccess) s = NGS_HIP_ERROR;
    }
    const hipError_t e2 = hipStreamEndCapture(cs, &graph);  // always ends the capture
    if (s == NGS_OK && e2 != hipSuccess) { e = e2; s = NGS_HIP_ERROR; }
  } else {
    s = NGS_HIP_ERROR;
  }
  prof_resume(prof);
  (void)hipStreamDestroy(cs);
  if (s != NGS_OK) {
    if (e != hipSuccess) ctx->last_hip = (int32_t)e;
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    ctx->last_hip = (int32_t)e;
    (void)hipGraphDestroy(graph);
    return NGS_HIP_ERROR;
  }
  ngs_score_graph* g = new ngs_score_graph;
  g->ctx = ctx;
  g->graph = graph;
  g->exec = exec;
  *out = g;
  return NGS_OK;
}

ngs_status ngs_score_graph_launch(ngs_score_graph* g, void* stream) {
  if (!g || !g->exec) return NGS_INVALID_ARG;
  NGS_TRY_HIP(g->ctx, hipSetDevice(g->ctx->device));
  NGS_TRY_HIP(g->ctx, hipGraphLaunch(g->exec, (hipStream_t)stream));
  return NGS_OK;
}

ngs_status ngs_score_graph_destroy(ngs_score_graph* g) {
  if (!g) return NGS_INVALID_ARG;
  (void)hipSetDevice(g->ctx->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
  return NGS_OK;
}

ngs_status ngs_set_tuning(ngs_ctx* ctx, const ngs_tuning* t) {
  if (!ctx || !t) return NGS_INVALID_ARG;
  if (t->ig_lanes_per_pixel != 0 && t->ig_lanes_per_pixel != 1 && t->ig_lanes_per_pixel != 2 &&
      t->ig_lanes_per_pixel != 4)
    return NGS_INVALID_ARG;
  if (t->ig_waves_per_simd != 0 && t->ig_waves_per_simd != 4) return NGS_INVALID_ARG;
  if (t->bin_chunk != 0 && (t->bin_chunk < 256 || t->bin_chunk > 8192 || (t->bin_chunk & (t->bin_chunk - 1))))
    return NGS_INVALID_ARG;
  if (t->groups_in_flight < 0 || t->groups_in_flight > 4) return NGS_INVALID_ARG;
  ctx->tuning = *t;
  return NGS_OK;
}

ngs_status ngs_get_tuning(const ngs_ctx* ctx, ngs_tuning* t) {
  if (!ctx || !t) return NGS_INVALID_ARG;
  *t = ctx->tuning;
  return NGS_OK;
}

ngs_status ngs_profile_enable(ngs_ctx* ctx, int32_t on) {
  if (!ctx) return NGS_INVALID_ARG;
  prof_enable(on != 0);
  return NGS_OK;
}

ngs_status ngs_profile_enable_class(ngs_ctx* ctx, int32_t id) {
  if (!ctx || id < 0 || id >= kProfKernels) return NGS_INVALID_ARG;
  prof_enable(true, id);
  return NGS_OK;
}

int32_t ngs_profile_kernels(void) { return kProfKernels; }

const char* ngs_profile_kernel_name(int32_t id) { return prof_name(id); }

ngs_status ngs_profile_read(ngs_ctx* ctx, int32_t id, double* total_ms, int64_t* launches) {
  if (!ctx || !total_ms || !launches || id < 0 || id >= kProfKernels) return NGS_INVALID_ARG;
  prof_read(id, total_ms, launches);
  return NGS_OK;
}

ngs_status ngs_render_backward(ngs_ctx* ctx, const ngs_scene* scene, const ngs_projected* proj,
                               const ngs_tile_lists* lists, const ngs_camera* cam, const ngs_raster_params* rp,
                               int32_t obj_eq2, const ngs_image_grad* grad_image, ngs_scene_grad* grad_scene,
                               void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !grad_image || !grad_scene) return NGS_INVALID_ARG;
  ngs_status s = check_scene(scene, true);
  if (s == NGS_OK) s = check_cam(cam, rp);
  if (s == NGS_OK) s = check_proj(proj);
  if (s == NGS_OK) s = check_lists(lists);
  if (s != NGS_OK) return s;
  const ngs_scene_grad& o = *grad_scene;
  if (!o.mean || !o.log_scale || !o.rot || !o.opacity_logit || !o.rgb || !o.obj_logit) return NGS_INVALID_ARG;
  if (!ws || ws_bytes < bwd_ws_bytes(scene->n, scene->k)) return NGS_WORKSPACE_TOO_SMALL;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  NGS_TRY_HIP(ctx, launch_render_backward(*scene, *proj, *lists, make_devcam(*cam, kTile), *rp, obj_eq2 ? 1 : 0,
                                          *grad_image, o, ws, (hipStream_t)stream));
  return NGS_OK;
}

// ---- learned view scorer ----------------------------------------------------------------

namespace {
bool sur_params_ok(const ngs_sur_params* p, bool need_bf16) {
  if (!p) return false;
  for (int l = 0; l < NGS_SUR_LAYERS; ++l)
    if (!p->w[l] || !p->b[l] || (need_bf16 && !p->w_bf16[l])) return false;
  return true;
}
}  // namespace

ngs_status ngs_sur_workspace_size(int32_t batch, size_t* bytes) {
  if (batch < 1 || !bytes) return NGS_INVALID_ARG;
  *bytes = sur_workspace_bytes(batch);
  return NGS_OK;
}

ngs_status ngs_sur_sync_bf16(ngs_ctx* ctx, const ngs_sur_params* params, void* stream) {
  if (!ctx || !sur_params_ok(params, true)) return NGS_INVALID_ARG;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  NGS_TRY_HIP(ctx, sur_sync_bf16(*params, (hipStream_t)stream));
  return NGS_OK;
}

ngs_status ngs_sur_forward(ngs_ctx* ctx, const ngs_sur_params* params, const float* x, int32_t batch, float* pred,
                           void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !sur_params_ok(params, true) || !x || !pred || batch < 1) return NGS_INVALID_ARG;
  if (!ws || ws_bytes < sur_workspace_bytes(batch)) return NGS_WORKSPACE_TOO_SMALL;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  NGS_TRY_HIP(ctx, sur_forward(*params, x, batch, pred, ws, (hipStream_t)stream));
  return NGS_OK;
}

ngs_status ngs_sur_backward(ngs_ctx* ctx, const ngs_sur_params* params, const float* x, int32_t batch,
                            const float* dpred, ngs_sur_params* grads, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !sur_params_ok(params, true) || !sur_params_ok(grads, false) || !dpred || batch < 1)
    return NGS_INVALID_ARG;
  if (!ws || ws_bytes < sur_workspace_bytes(batch)) return NGS_WORKSPACE_TOO_SMALL;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  NGS_TRY_HIP(ctx, sur_backward(*params, x, batch, dpred, *grads, ws, (hipStream_t)stream));
  return NGS_OK;
}

ngs_status ngs_sur_mse(ngs_ctx* ctx, const float* pred, const float* target, int32_t batch, float* dpred, float* loss,
                       void* stream) {
  if (!ctx || !pred || !target || !dpred || batch < 1) return NGS_INVALID_ARG;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  NGS_TRY_HIP(ctx, sur_mse(pred, target, batch, dpred, loss, (hipStream_t)stream));
  return NGS_OK;
}

ngs_status ngs_sur_adam(ngs_ctx* ctx, ngs_sur_params* params, const ngs_sur_params* g, ngs_sur_params* m,
                        ngs_sur_params* v, float lr, float beta1, float beta2, float eps, int32_t step, void* stream) {
  if (!ctx || !sur_params_ok(params, true) || !sur_params_ok(g, false) || !sur_params_ok(m, false) ||
      !sur_params_ok(v, false) || step < 1)
    return NGS_INVALID_ARG;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  NGS_TRY_HIP(ctx, sur_adam(*params, *g, *m, *v, lr, beta1, beta2, eps, step, (hipStream_t)stream));
  return NGS_OK;
}

ngs_status ngs_sur_features(ngs_ctx* ctx, const ngs_image* img, int32_t width, int32_t height, int32_t k,
                            float depth_scale, float* x, int32_t batch, int32_t index, void* stream) {
  if (!ctx || !img || !img->depth || !img->t_final || !img->argmax_id || !img->mean_conf || !x) return NGS_INVALID_ARG;
  if (width != NGS_SUR_IN_W || height != NGS_SUR_IN_H || k < 1 || !(depth_scale > 0.f) || index < 0 ||
      index >= batch)
    return NGS_INVALID_ARG;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  NGS_TRY_HIP(ctx, sur_features(*img, width, height, k, depth_scale, x, batch, index, 1, 0, (hipStream_t)stream));
  return NGS_OK;
}

ngs_status ngs_sur_novelty(ngs_ctx* ctx, const ngs_scene* scene, const ngs_hessian* h, float lambda_prior,
                           float* out, void* stream) {
  if (!ctx || !out || !(lambda_prior > 0.f)) return NGS_INVALID_ARG;
  ngs_status s = check_scene(scene, true);
  if (s != NGS_OK) return s;
  if (h && (!h->slot_of || !h->logdet || h->capacity < 1 || h->k != scene->k)) return NGS_INVALID_ARG;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  NGS_TRY_HIP(ctx, sur_novelty(*scene, h, lambda_prior, out, (hipStream_t)stream));
  return NGS_OK;
}

ngs_status ngs_sur_render_features(ngs_ctx* ctx, const ngs_scene* scene, const ngs_camera* cams, int32_t n_views,
                                   const ngs_raster_params* rp, const float* weight, float depth_scale, float* x,
                                   const ngs_dims* dims, void* ws, size_t ws_bytes, void* stream) {
  if (!ctx || !cams || n_views < 1 || !x || !dims || !(depth_scale > 0.f)) return NGS_INVALID_ARG;
  if (dims->n != scene->n || dims->k != scene->k || dims->max_pairs < 1) return NGS_INVALID_ARG;
  ngs_status s = check_scene(scene, true);
  if (s != NGS_OK) return s;
  for (int v = 0; v < n_views; ++v) {
    s = check_cam(&cams[v], rp);
    if (s != NGS_OK) return s;
    if (cams[v].width != NGS_SUR_IN_W || cams[v].height != NGS_SUR_IN_H) return NGS_INVALID_ARG;
  }
  size_t need = 0;
  s = ngs_workspace_size(4, dims, &need);
  if (s != NGS_OK) return s;
  if (!ws || ws_bytes < need) return NGS_WORKSPACE_TOO_SMALL;
  hipStream_t st = (hipStream_t)stream;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  // Views go in groups of G: a group is projected and binned on a context stream with one
  // launch per kernel and sub-group of at most 16 views (grid.y = view), then one render launch
  // composites the whole group (grid.y = view) and one launch writes its feature channels,
  // both on `stream`. Groups alternate between two halves of the buffer sets and two streams,
  // so binning of the next group overlaps the render of this one.
  const int G = std::max(1, std::min(views_in_flight(dims, kMaxFeatureGroup), n_views));
  s = ensure_lanes(ctx, 2);
  if (s != NGS_OK) return s;
  int32_t* sticky = static_cast<int32_t*>(ws);
  NGS_TRY_HIP(ctx, hipMemsetAsync(sticky, 0, kIgHeader, st));
  const size_t per = (need - kIgHeader) / (2 * (size_t)views_in_flight(dims, kMaxFeatureGroup));
  char* base = static_cast<char*>(ws) + kIgHeader;
  const size_t fixed = al(batch_fixed_bytes(scene->n, dims->max_pairs));
  NGS_TRY_HIP(ctx, hipEventRecord(ctx->fork, st));
  for (int i = 0; i < 2; ++i) NGS_TRY_HIP(ctx, hipStreamWaitEvent(ctx->lanes[i], ctx->fork, 0));
  const RasterConst rc = make_raster(*rp);
  ngs_scene ws_scene = *scene;  // the render averages `weight` where it would average kappa
  if (weight) ws_scene.kappa = const_cast<float*>(weight);
  std::vector<DevCam> dcs(n_views);
  for (int v = 0; v < n_views; ++v) dcs[v] = make_devcam(cams[v], kTile);
  for (int q = 0, v0 = 0; v0 < n_views; ++q, v0 += G) {
    const int g = std::min(G, n_views - v0);
    const int half = q & 1;
    hipStream_t ls = ctx->lanes[half];
    if (q >= 2) NGS_TRY_HIP(ctx, hipStreamWaitEvent(ls, ctx->half_done[half], 0));
    char* first = base + (size_t)(half * G) * per;
    for (int s0 = 0; s0 < g; s0 += kMaxGroup) {
      const int sg = std::min(kMaxGroup, g - s0);
      BatchWs b = batch_carve(first + (size_t)s0 * per, fixed, scene->n, dims->max_pairs);
      b.proj.splat = nullptr;  // the render reads the planes, not the walk records
      const BinWs bw = bin_ws_carve(b.bin, scene->n, dims->max_pairs);
      const Group Gs = make_group(&dcs[v0 + s0], sg, per);
      NGS_TRY_HIP(ctx, launch_project(*scene, Gs, *rp, b.proj, ls));
      NGS_TRY_HIP(ctx, bin_count_pairs(b.proj, scene->n, bw, ls, sg, per));
      NGS_TRY_HIP(ctx, bin_emit_and_sort(b.proj, scene->n, Gs, bw, b.lists, sticky, nullptr, ls));
    }
    NGS_TRY_HIP(ctx, hipEventRecord(ctx->lane_done[half], ls));
    NGS_TRY_HIP(ctx, hipStreamWaitEvent(st, ctx->lane_done[half], 0));
    const BatchWs b0 = batch_carve(first, fixed, scene->n, dims->max_pairs);
    const ngs_image img0 = feat_img_carve(first + fixed);
    const DevCam dc0 = dcs[v0];  // every view is 80 x 60: one tile grid
    NGS_TRY_HIP(ctx, launch_render_views(ws_scene, b0.proj, b0.lists, dc0, rc, img0, g, per, st));
    NGS_TRY_HIP(ctx, sur_features(img0, NGS_SUR_IN_W, NGS_SUR_IN_H, scene->k, depth_scale, x, n_views, v0, g, per,
                                  st));
    NGS_TRY_HIP(ctx, hipEventRecord(ctx->half_done[half], st));
  }
  int64_t of = 0;
  s = read_i64(ctx, sticky, 4, st, &of);
  if (s != NGS_OK) return s;
  return of ? NGS_CAPACITY : NGS_OK;
}

ngs_status ngs_gemm_bf16(ngs_ctx* ctx, int32_t trans_a, int32_t trans_b, int32_t m, int32_t n, int32_t k,
                         const uint16_t* a, int32_t lda, const uint16_t* b, int32_t ldb, float* c, int32_t ldc,
                         float beta, void* stream) {
  if (!ctx || !a || !b || !c || m < 0 || n < 0 || k < 0) return NGS_INVALID_ARG;
  if (ldc < n || lda < (trans_a ? m : k) || ldb < (trans_b ? k : n)) return NGS_INVALID_ARG;
  NGS_TRY_HIP(ctx, hipSetDevice(ctx->device));
  NGS_TRY_HIP(ctx, sur_gemm(trans_a != 0, trans_b != 0, m, n, k, a, lda, b, ldb, c, ldc, beta, (hipStream_t)stream));
  return NGS_OK;
}

}  // extern "C"
