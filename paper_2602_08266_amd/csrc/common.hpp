// common.hpp -- internal declarations shared by the HIP translation units of libngs.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstddef>
#include <cstdint>
#include <type_traits>

#include "../../include/ngs.h"
#include "../../include/ngs_surrogate.h"

namespace ngs {

constexpr int kTile = 16;
constexpr int kTilePix = kTile * kTile;  // one workgroup of 256 lanes per tile
constexpr int kWave = 64;
constexpr int kNGeo = 11;                // mu 3, log-scale 3, quaternion 4, opacity logit 1
constexpr int kNScreen = 6;              // m_x, m_y, Q_xx, Q_xy, Q_yy, opacity logit

// Screen-space statistics of one touched Gaussian (per view), FP32, accumulated over its
// contributing pixels:
//   Y_rgb  sym 6x6  sum |w_rgb|^2 y y^T
//   X_rgb  6x3      sum a y w_rgb^T
//   Y_d    sym 7x7  sum e e^T, e = (w_d y, a)         (e_6 e_6 = sum a^2)
//   Y_o    sym 6x6  sum |w_o|^2 y y^T
//   m1     6        sum a T y
//   Z_o    6 x k    sum (a / (1 - alpha)) y S~^T      (S~: object suffix incl. Eq. 2 residual)
// y = d alpha / d(m_x, m_y, Q_xx, Q_xy, Q_yy, l), a = alpha T, w = d out / d alpha.
constexpr int kStatYrgb = 0;
constexpr int kStatXrgb = 21;
constexpr int kStatYd = 39;
constexpr int kStatYo = 67;
constexpr int kStatM1 = 88;
constexpr int kStatScalar = 94;          // first index of Z_o
inline __host__ __device__ int stat_len(int k) { return kStatScalar + 6 * k; }

inline __host__ __device__ int tri_len(int l) { return l * (l + 1) / 2; }
// packed upper triangle, row-major: (i, j) with i <= j
inline __host__ __device__ int tri_idx(int i, int j, int l) { return i * l - (i * (i - 1)) / 2 + (j - i); }

// Quadratic form q = d^T Q d of the conic and the unclamped opacity sigma exp(-q / 2),
// evaluated without FMA contraction so that every kernel that re-walks a tile takes the
// same cut-off and alpha decisions bit for bit.
__device__ __forceinline__ float conic_q(float qa, float qb, float qc, float dx, float dy) {
#pragma clang fp contract(off)
  return qa * dx * dx + 2.f * qb * dx * dy + qc * dy * dy;
}
__device__ __forceinline__ float gauss_alpha(float op, float q) {
#pragma clang fp contract(off)
  return op * __expf(-0.5f * q);
}
__device__ __forceinline__ float transmit(float T, float alpha) {
#pragma clang fp contract(off)
  return T * (1.f - alpha);
}

// Half-extents of the conic's ellipse q <= cut along x and y (x within m_x +- sqrt(cut *
// Sigma_xx), Sigma = Q^-1), widened by 1% + 0.05 px so that FP32 rounding never culls a
// pixel with q <= cut. Used to skip, per wavefront, entries that cannot reach any of its
// pixels; a degenerate conic is never culled.
__device__ __forceinline__ void conic_extent(float qa, float qb, float qc, float cut, float* hx, float* hy) {
  const float det = qa * qc - qb * qb;
  if (!(det > 0.f) || !(qa > 0.f) || !(qc > 0.f)) {
    *hx = __builtin_inff();
    *hy = __builtin_inff();
    return;
  }
  *hx = sqrtf(cut * qc / det) * 1.01f + 0.05f;
  *hy = sqrtf(cut * qa / det) * 1.01f + 0.05f;
}

// Whether the ellipse q <= cut of a conic centred at (mx, my) can reach a pixel centre of the
// strip [sx0, sx1] x [sy0, sy1] (pixel-centre bounds): the least q over the rectangle (0 when it
// holds the centre; else on an edge, where q is a 1D quadratic minimised at a clamped point)
// against the cut-off. The slack (1e-5 of the largest magnitude the three terms of q take on
// the rectangle, plus 0.1 % of the cut-off) exceeds the FP32 rounding of q here and at any
// pixel centre, so a pixel whose own q <= cut is never dropped. A degenerate conic always
// reaches. The walks use it on top of the box test: an entry it rejects would be passed over at
// every pixel of the strip.
__device__ __forceinline__ bool ellipse_meets(float mx, float my, float qa, float qb, float qc, float sx0, float sx1,
                                              float sy0, float sy1, float cut) {
  const float dx0 = sx0 - mx, dx1 = sx1 - mx, dy0 = sy0 - my, dy1 = sy1 - my;
  if (dx0 <= 0.f && dx1 >= 0.f && dy0 <= 0.f && dy1 >= 0.f) return true;
  if (!(qa > 0.f) || !(qc > 0.f)) return true;
  const float ia = __builtin_amdgcn_rcpf(qa), ic = __builtin_amdgcn_rcpf(qc);
  const auto q = [&](float x, float y) { return qa * x * x + 2.f * qb * x * y + qc * y * y; };
  float m = q(dx0, fminf(fmaxf(-qb * dx0 * ic, dy0), dy1));
  m = fminf(m, q(dx1, fminf(fmaxf(-qb * dx1 * ic, dy0), dy1)));
  m = fminf(m, q(fminf(fmaxf(-qb * dy0 * ia, dx0), dx1), dy0));
  m = fminf(m, q(fminf(fmaxf(-qb * dy1 * ia, dx0), dx1), dy1));
  const float ax = fmaxf(fabsf(dx0), fabsf(dx1)), ay = fmaxf(fabsf(dy0), fabsf(dy1));
  const float mag = qa * ax * ax + 2.f * fabsf(qb) * ax * ay + qc * ay * ay;
  return m <= cut * 1.001f + 1e-5f * mag;
}

struct DevCam {
  float R[9], t[3], fx, fy, cx, cy;
  int width, height, tiles_x, tiles_y;
};

// Several views in one launch: grid.y is the view of the group, view v's buffers lie v * vs
// bytes past the pointers passed (buffer sets of equal layout, one after another), and its
// camera is cams.c[v]. Grids are sized for the largest view of the group; blocks past a view's
// own extent leave at once. A single view is the group {1, 0, {cam}}.
constexpr int kMaxGroup = 16;
struct GroupCams {
  DevCam c[kMaxGroup];
};
struct GroupDims {  // tile grid of each view (what the binning kernels need of the cameras)
  int tx[kMaxGroup], ty[kMaxGroup];
};
struct Group {
  int g = 1;
  size_t vs = 0;
  GroupCams cams;
  GroupDims dims;
  int max_tiles_x = 0, max_tiles_y = 0, max_ntiles = 0, max_width = 0, max_height = 0;
};

// OR of a 32-bit value over the wavefront, by DPP moves (no LDS round trips): an inclusive OR
// scan within each row of 16 lanes (shifts 1, 2, 4, 8), then the row totals broadcast into
// the later rows (row_bcast 15 and 31); lane 63 ends with the OR of all 64 lanes.
__device__ __forceinline__ uint32_t wave_or32(uint32_t x) {
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
  x |= (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// This block's view of a per-view pointer.
template <class T>
__device__ __forceinline__ T* vp(T* p, size_t vs) {
  using Byte = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return p ? reinterpret_cast<T*>(reinterpret_cast<Byte*>(p) + (size_t)blockIdx.y * vs) : p;
}

inline Group make_group(const DevCam* cams, int g, size_t vs) {
  Group G;
  G.g = g;
  G.vs = vs;
  for (int i = 0; i < kMaxGroup; ++i) G.dims.tx[i] = G.dims.ty[i] = 0;
  for (int i = 0; i < g; ++i) {
    G.cams.c[i] = cams[i];
    G.dims.tx[i] = cams[i].tiles_x;
    G.dims.ty[i] = cams[i].tiles_y;
    G.max_tiles_x = std::max(G.max_tiles_x, cams[i].tiles_x);
    G.max_tiles_y = std::max(G.max_tiles_y, cams[i].tiles_y);
    G.max_ntiles = std::max(G.max_ntiles, cams[i].tiles_x * cams[i].tiles_y);
    G.max_width = std::max(G.max_width, cams[i].width);
    G.max_height = std::max(G.max_height, cams[i].height);
  }
  return G;
}

inline Group single_group(const DevCam& cam) { return make_group(&cam, 1, 0); }

inline DevCam make_devcam(const ngs_camera& c, int tile) {
  DevCam d;
  for (int i = 0; i < 9; ++i) d.R[i] = c.R[i];
  for (int i = 0; i < 3; ++i) d.t[i] = c.t[i];
  d.fx = c.fx; d.fy = c.fy; d.cx = c.cx; d.cy = c.cy;
  d.width = c.width; d.height = c.height;
  d.tiles_x = (c.width + tile - 1) / tile;
  d.tiles_y = (c.height + tile - 1) / tile;
  return d;
}

struct RasterConst {
  float z_near, eps2d, cutoff_q, alpha_min, alpha_max, t_min;
};

inline RasterConst make_raster(const ngs_raster_params& r) {
  return RasterConst{r.z_near, r.eps2d, r.cutoff_q, r.alpha_min, r.alpha_max, r.t_min};
}

// Kernel classes of the optional event profiler (prof.hip). ProfScope brackets one launch.
enum ProfId {
  kProfPrepare = 0, kProfProject, kProfDepthHist, kProfDepthScan, kProfDepthScatter, kProfCountScan,
  kProfEmit, kProfRanges, kProfKeys64, kProfRender, kProfIgTiles, kProfIgFinalize, kProfHessianLogdet,
  kProfCombine, kProfFill, kProfTileHist, kProfTileScan, kProfTileScatter, kProfIgAssign, kProfBwdTiles, kProfBwdParams, kProfSurGemm, kProfSurForward,
  kProfSurBackward, kProfIgFront, kProfKernels
};
class ProfScope {
 public:
  ProfScope(int id, hipStream_t st);
  ~ProfScope();
 private:
  int id_;
  hipStream_t st_;
  void* a_;
};
// only >= 0 restricts the timing to that kernel class (fewer events on the streams)
void prof_enable(bool on, int only = -1);
// Pause timing without clearing what was recorded (graph capture records no profiling events).
bool prof_suspend();
void prof_resume(bool on);
void prof_read(int id, double* ms, int64_t* count);
const char* prof_name(int id);

// Launchers implemented in the .hip files (stream-ordered, no synchronisation).
hipError_t launch_prepare_scene(const ngs_scene& s, const ngs_ig_params& ig, hipStream_t st);
// tight: the tile rects of the information walks (only tiles with a pixel centre in the
// ellipse's box; the lists then hold exactly the entries a walk can take); else the rects of
// the 3DGS pipeline (box of the 3-sigma circle of the largest eigenvalue). tflag (per view at
// the group's stride, cleared beforehand): also flag the tiles that the rects of weighted
// Gaussians reach (what launch_ig_assign does after a projection without it).
hipError_t launch_project(const ngs_scene& s, const Group& G, const ngs_raster_params& rp,
                          const ngs_projected& out, hipStream_t st, int tight = 0, int32_t* tflag = nullptr);
// Adds the view's pair count (sum of p.count over n Gaussians) to *total (device).
hipError_t launch_sum_counts(const ngs_projected& p, int n, int64_t* total, hipStream_t st);

// Radix-sort building blocks (sort.hip).
struct SortWs {
  uint32_t* hist;       // [256][max blocks]
  uint32_t* rowtot;     // [256]
  size_t max_blocks;
};
size_t sort_blocks_for(size_t n);
hipError_t radix_sort_pairs(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_a,
                            uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, size_t n,
                            int begin_bit, int end_bit, const SortWs& ws, hipStream_t st,
                            uint32_t** keys_out, uint32_t** vals_out, int prof_base,
                            const void* rec_in = nullptr, void* rec_sorted = nullptr, int g = 1, size_t vs = 0);
hipError_t launch_iota(uint32_t* v, size_t n, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* v, uint32_t x, size_t n, hipStream_t st, int g = 1, size_t vs = 0);
hipError_t launch_fill_i32(int32_t* v, int32_t x, size_t n, hipStream_t st);
// Device-to-device copy of n 32-bit words by a kernel (graph-capturable like the fills: the
// scoring path records no memset or memcpy nodes).
hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, size_t n, hipStream_t st);

// Binning (bin.hip).
struct BinWs {
  uint32_t* dkeys[2];   // depth keys ping-pong [n]
  uint32_t* dvals[2];   // gids ping-pong [n]
  uint64_t* m_total;    // [1] the view's pair count M
  uint64_t* blocksum;   // partial sums of the tile counts
  uint32_t* phist;      // level 1: row entries per (row, block) [4096][ceil(n / 512)]
  uint32_t* ptot;       // pairs per tile [4096]
  SortWs sort;
  uint2* rl;            // level 1 output: {gid, x0 | w << 16} per (row, Gaussian) [max_pairs]
  int16_t* rect_sorted; // [n][4] the tile rects in depth order (written by the last sort pass)
  uint32_t* hist2;      // level 2: pairs per (tile, chunk), row by row
  uint32_t *rtot, *rstart, *nch, *cp;  // per row: entries, start, chunks, chunk prefix [4097]
  uint32_t* meta;       // M, entries per chunk, chunks, overflow
  unsigned long long* rkm;  // [NGS_MAX_TILES][2] per row: its wanted tiles (with keep flags)
};
size_t bin_ws_bytes(int64_t n, int64_t max_pairs);
BinWs bin_ws_carve(void* ws, int64_t n, int64_t max_pairs);
hipError_t bin_count_pairs(const ngs_projected& p, int n, const BinWs& w, hipStream_t st, int g = 1, size_t vs = 0);
// Pairs beyond out.capacity are not written: the ranges are left empty and *overflow (may
// be NULL) is raised; stats[1] (may be NULL) accumulates the pair count. keep (may be NULL:
// every tile) flags the tiles whose lists are wanted: the others get empty ranges and none of
// their gids is written, while the wanted lists and M stay those of the full binning.
// chunk2: least row entries per level-2 chunk (0 = 512): longer chunks write longer runs per
// tile and leave fewer partly written lines, shorter ones spread the scatter over more blocks.
hipError_t bin_emit_and_sort(const ngs_projected& p, int n, const Group& G, const BinWs& w,
                             const ngs_tile_lists& out, int32_t* overflow, int64_t* stats, hipStream_t st,
                             const int32_t* keep = nullptr, int chunk2 = 0);

// Rendering (render.hip).
hipError_t launch_render(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l,
                         const DevCam& cam, const RasterConst& rc, const ngs_image& img,
                         hipStream_t st);
// Views of one size in one launch (grid.y = view); view v's projection, lists and images lie
// v * stride bytes past those passed.
hipError_t launch_render_views(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l, const DevCam& cam,
                               const RasterConst& rc, const ngs_image& img, int views, size_t stride,
                               hipStream_t st);

// Information gain (info_gain.hip, finalize.hip).
struct IgWs {
  float* acc;           // [max_slots][astride] per-view screen statistics, slot-major
  int astride;          // stat_len(k) rounded up to 16 floats
  int32_t* slot_of;     // [n] per-view slot, -1 for Gaussians that are not reduced (-1 between views)
  int32_t* gid_of;      // [max_slots]
  int32_t* n_slots;     // [1]
  int32_t* overflow;    // [1]
  double* pmat;         // [max_slots][7][11] chain-rule matrix P of each slot (finalize)
  int32_t* tflag;       // [NGS_MAX_TILES] tiles reached by a weighted Gaussian's rect
  float* pix_t;         // [NGS_MAX_TILES][256] final transmittance per pixel (pass 1)
  int32_t* pix_last;    // [NGS_MAX_TILES][256] last contributor's list position, -1 for none
  int2* wave_range;     // [NGS_MAX_TILES][4] per 16 x 4 strip: first weighted and last contributor
  int64_t max_slots;
};
int ig_stat_stride(int64_t k);
size_t ig_ws_fixed_bytes(int64_t n);  // the part that does not grow with the slots
size_t ig_ws_bytes(int64_t n, int64_t k, int64_t max_slots);
IgWs ig_ws_carve(void* ws, int64_t n, int64_t k, int64_t max_slots);
// lpp: lanes per pixel of the tile kernel (1, 2 or 4; 0 = the default for k); it sets the
// workgroup size and the rows per LDS reduction round. ig_lpp_valid tells which k allow which.
// waves: waves per SIMD of the back pass (0 = default, 4 = the two-workgroups-per-CU variant;
// see ig_waves_valid).
hipError_t launch_ig_tiles(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l,
                           const Group& G, const RasterConst& rc, const ngs_ig_params& ig,
                           const IgWs& w, int64_t* stats, int lpp, hipStream_t st, int waves = 0);
// The two halves of launch_ig_tiles: with a target object the flags of the tiles that a
// weighted Gaussian's rect reaches (see ig_tile_flags; needed before the filtered binning),
// then the walk (front pass, slots of the contributing weighted Gaussians, back pass).
// launch_ig_reset_slots sets every Gaussian's slot of a fresh workspace to -1 (the front pass
// claims slots from -1; the finalisation sets the claimed ones back).
hipError_t launch_ig_reset_slots(const IgWs& w, int64_t n, hipStream_t st);
hipError_t launch_ig_assign(const ngs_scene& s, const ngs_projected& p, const Group& G, const ngs_ig_params& ig,
                            const IgWs& w, hipStream_t st);
// The first half of launch_ig_assign alone (slot counter, overflow flag and tile flags
// cleared), for a projection that flags the tiles itself.
hipError_t launch_ig_clear(const ngs_ig_params& ig, const IgWs& w, const Group& G, hipStream_t st);
hipError_t launch_ig_walk(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l, const Group& G,
                          const RasterConst& rc, const ngs_ig_params& ig, const IgWs& w, int64_t* stats, int lpp,
                          hipStream_t st, int waves = 0);
// Tile flags of w when launch_ig_assign fills them (a target object), else nullptr.
const int32_t* ig_tile_flags(const ngs_ig_params& ig, const IgWs& w);
bool ig_lpp_valid(int64_t k, int lpp);
bool ig_waves_valid(int64_t k, int lpp, int waves);
// ig_out: three gains per view of the group, view after view (scoring); accumulation takes
// a group of one view.
hipError_t launch_ig_finalize(const ngs_scene& s, const Group& G, const ngs_raster_params& rp,
                              const ngs_ig_params& ig, const IgWs& w, ngs_hessian* h,
                              double* ig_out, int64_t* stats, int32_t* sticky, hipStream_t st);
hipError_t launch_hessian_logdet(ngs_hessian* h, int32_t n_slots, float lambda_prior, hipStream_t st);
// Eq. 10 normalisers (and, for the trace criterion, S_f) from the training views' raw gains.
hipError_t launch_train_normalisers(const ngs_hessian& h, int n, int k, const ngs_ig_params& ig, const double* ig_train,
                                    int n_train, double* norm, double* trace_total, hipStream_t st);
// Backward rasterizer (backward.hip).
size_t bwd_ws_bytes(int64_t n, int64_t k);
hipError_t launch_render_backward(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l,
                                  const DevCam& cam, const ngs_raster_params& rp, int obj_eq2,
                                  const ngs_image_grad& gi, const ngs_scene_grad& out, void* ws, hipStream_t st);
// Learned view scorer (surrogate.hip).
size_t sur_workspace_bytes(int batch);
hipError_t sur_gemm(bool ta, bool tb, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                    float* C, int ldc, float beta, hipStream_t st);
hipError_t sur_sync_bf16(const ngs_sur_params& p, hipStream_t st);
hipError_t sur_forward(const ngs_sur_params& p, const float* x, int B, float* pred, void* ws, hipStream_t st);
hipError_t sur_backward(const ngs_sur_params& p, const float* x, int B, const float* dpred, const ngs_sur_params& g,
                        void* ws, hipStream_t st);
hipError_t sur_mse(const float* pred, const float* target, int B, float* dpred, float* loss, hipStream_t st);
hipError_t sur_adam(const ngs_sur_params& p, const ngs_sur_params& g, const ngs_sur_params& m,
                    const ngs_sur_params& v, float lr, float b1, float b2, float eps, int step, hipStream_t st);
hipError_t sur_novelty(const ngs_scene& s, const ngs_hessian* h, float lambda, float* out, hipStream_t st);
hipError_t sur_features(const ngs_image& img, int W, int H, int k, float depth_scale, float* x, int B, int index,
                        int views, size_t set_stride, hipStream_t st);
hipError_t launch_score_combine(const double* ig_raw, int n_views, double n0, double n1, double n2,
                                const double* nf_dev, const ngs_ig_params& ig, float* scores, int32_t* best,
                                hipStream_t st);

}  // namespace ngs
