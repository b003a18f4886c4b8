// render.hip -- front-to-back compositing of colour, depth and the object vector.
//
// One 256-lane workgroup per 16x16 tile, one lane per pixel (4 wavefronts of 4 pixel rows).
// The tile's depth-sorted list is staged through LDS in batches of kBatch Gaussians
// (SoA scalars plus the k-long probability rows). A pixel leaves the walk at the first
// Gaussian that would drop its transmittance below t_min; a wavefront stops issuing once
// all its lanes have left, and the workgroup stops loading batches once all 256 have.
// Several views of one size can share a launch (grid.y = view): their per-view buffers
// (projection, lists, images) sit at a fixed byte stride from the first view's.
#include "common.hpp"

namespace ngs {
namespace {

constexpr int kBatch = 64;

template <int KP>
__global__ __launch_bounds__(kTilePix) void k_render(int n, int k, const uint32_t* __restrict__ gids,
                                                     const uint32_t* __restrict__ ranges, DevCam cam, RasterConst rc,
                                                     const float* __restrict__ mean2d, const float* __restrict__ conic,
                                                     const float* __restrict__ depth, const float* __restrict__ opacity,
                                                     const float* __restrict__ rgb, const float* __restrict__ prob,
                                                     const float* __restrict__ kappa, float* __restrict__ out_rgb,
                                                     float* __restrict__ out_depth, float* __restrict__ out_obj,
                                                     float* __restrict__ out_t, float* __restrict__ out_conf,
                                                     int32_t* __restrict__ out_id, int32_t* __restrict__ out_nc,
                                                     size_t set_stride) {
  if (blockIdx.y) {
    const size_t so = (size_t)blockIdx.y * set_stride;
    gids = (const uint32_t*)((const char*)gids + so);
    ranges = (const uint32_t*)((const char*)ranges + so);
    mean2d = (const float*)((const char*)mean2d + so);
    conic = (const float*)((const char*)conic + so);
    depth = (const float*)((const char*)depth + so);
    if (out_rgb) out_rgb = (float*)((char*)out_rgb + so);
    if (out_depth) out_depth = (float*)((char*)out_depth + so);
    if (out_obj) out_obj = (float*)((char*)out_obj + so);
    if (out_t) out_t = (float*)((char*)out_t + so);
    if (out_conf) out_conf = (float*)((char*)out_conf + so);
    if (out_id) out_id = (int32_t*)((char*)out_id + so);
    if (out_nc) out_nc = (int32_t*)((char*)out_nc + so);
  }
  __shared__ float s_mx[kBatch], s_my[kBatch], s_qa[kBatch], s_qb[kBatch], s_qc[kBatch], s_op[kBatch];
  __shared__ float s_z[kBatch], s_r[kBatch], s_g[kBatch], s_b[kBatch], s_kap[kBatch], s_hx[kBatch], s_hy[kBatch];
  __shared__ float s_p[kBatch][KP];
  const int ntiles = cam.tiles_x * cam.tiles_y;
  const int tile = blockIdx.x;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int px = tx * kTile + (threadIdx.x & (kTile - 1));
  const int py = ty * kTile + (threadIdx.x / kTile);
  const bool inside = px < cam.width && py < cam.height;
  const float fxp = (float)px + 0.5f, fyp = (float)py + 0.5f;
  const uint32_t start = ranges[tile], end = ranges[ntiles + tile];
  // pixel-centre bounds of this wavefront's 16 x 4 strip
  const float sx0 = (float)(tx * kTile) + 0.5f, sx1 = sx0 + (float)(kTile - 1);
  const float sy0 = (float)(ty * kTile + (int)(threadIdx.x / kWave) * (kWave / kTile)) + 0.5f;
  const float sy1 = sy0 + (float)(kWave / kTile - 1);
  float T = 1.f, C0 = 0.f, C1 = 0.f, C2 = 0.f, D = 0.f, kb = 0.f;
  float Op[KP];
#pragma unroll
  for (int c = 0; c < KP; ++c) Op[c] = 0.f;
  int nc = 0;
  bool done = !inside;
  for (uint32_t b0 = start; b0 < end; b0 += kBatch) {
    if (__syncthreads_and(done)) break;
    const int cnt = (int)min((uint32_t)kBatch, end - b0);
    if ((int)threadIdx.x < cnt) {
      const uint32_t g = gids[b0 + threadIdx.x];
      const int j = threadIdx.x;
      s_mx[j] = mean2d[g]; s_my[j] = mean2d[n + g];
      s_qa[j] = conic[g]; s_qb[j] = conic[n + g]; s_qc[j] = conic[2 * n + g];
      s_op[j] = opacity[g]; s_z[j] = depth[g];
      s_r[j] = rgb[g]; s_g[j] = rgb[n + g]; s_b[j] = rgb[2 * n + g];
      s_kap[j] = kappa[g];
      conic_extent(s_qa[j], s_qb[j], s_qc[j], rc.cutoff_q, &s_hx[j], &s_hy[j]);
    }
    for (int idx = threadIdx.x; idx < cnt * KP; idx += kTilePix) {
      const int j = idx / KP, c = idx % KP;
      s_p[j][c] = (c < k) ? prob[(size_t)gids[b0 + j] * k + c] : 0.f;
    }
    __syncthreads();
    // entries whose ellipse can reach this wavefront's strip (lane l tests entry l)
    const int l = (int)(threadIdx.x % kWave);
    const bool reach = l < cnt && s_mx[l] + s_hx[l] >= sx0 && s_mx[l] - s_hx[l] <= sx1 &&
                       s_my[l] + s_hy[l] >= sy0 && s_my[l] - s_hy[l] <= sy1;
    uint64_t live = __ballot(reach);
    if (!done) {
      while (live) {
        const int j = __ffsll((unsigned long long)live) - 1;
        live &= live - 1;
        const float dx = fxp - s_mx[j], dy = fyp - s_my[j];
        const float q = conic_q(s_qa[j], s_qb[j], s_qc[j], dx, dy);
        if (q > rc.cutoff_q) continue;
        const float alpha = fminf(rc.alpha_max, gauss_alpha(s_op[j], q));
        if (alpha < rc.alpha_min) continue;
        const float Tn = transmit(T, alpha);
        if (Tn < rc.t_min) { done = true; break; }
        const float a = alpha * T;
        C0 += s_r[j] * a; C1 += s_g[j] * a; C2 += s_b[j] * a;
        D += s_z[j] * a;
        kb += s_kap[j] * a;
#pragma unroll
        for (int c = 0; c < KP; ++c) Op[c] += s_p[j][c] * a;
        T = Tn;
        ++nc;
      }
    }
  }
  if (!inside) return;
  const size_t HW = (size_t)cam.width * cam.height;
  const size_t pix = (size_t)py * cam.width + px;
  if (out_rgb) { out_rgb[pix] = C0; out_rgb[HW + pix] = C1; out_rgb[2 * HW + pix] = C2; }
  if (out_depth) out_depth[pix] = D;
  if (out_t) out_t[pix] = T;
  if (out_nc) out_nc[pix] = nc;
  if (out_conf) out_conf[pix] = nc ? kb / (1.f - T) : 0.f;
  // Eq. 2: the residual 1 - sum_k O'_k goes to the background channel 0.
  float so = 0.f;
#pragma unroll
  for (int c = 0; c < KP; ++c) so += Op[c];
  Op[0] += 1.f - so;
  int am = 0;
  float best = Op[0];
#pragma unroll
  for (int c = 1; c < KP; ++c)
    if (c < k && Op[c] > best) { best = Op[c]; am = c; }
  if (out_id) out_id[pix] = am;
  if (out_obj)
#pragma unroll
    for (int c = 0; c < KP; ++c)
      if (c < k) out_obj[c * HW + pix] = Op[c];
}

template <int KP>
hipError_t launch_render_k(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l, const DevCam& cam,
                           const RasterConst& rc, const ngs_image& img, int views, size_t stride, hipStream_t st) {
  const int ntiles = cam.tiles_x * cam.tiles_y;
  ProfScope ps(kProfRender, st);
  hipLaunchKernelGGL(k_render<KP>, dim3(ntiles, views), dim3(kTilePix), 0, st, s.n, s.k, l.gids, l.ranges, cam, rc,
                     p.mean2d, p.conic, p.depth, s.opacity, s.rgb, s.prob, s.kappa, img.rgb, img.depth, img.obj,
                     img.t_final, img.mean_conf, img.argmax_id, img.n_contrib, stride);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_render_views(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l, const DevCam& cam,
                               const RasterConst& rc, const ngs_image& img, int views, size_t stride,
                               hipStream_t st) {
  if (views < 1) return hipSuccess;
  if (s.k <= 4) return launch_render_k<4>(s, p, l, cam, rc, img, views, stride, st);
  if (s.k <= 8) return launch_render_k<8>(s, p, l, cam, rc, img, views, stride, st);
  if (s.k <= 16) return launch_render_k<16>(s, p, l, cam, rc, img, views, stride, st);
  if (s.k <= 32) return launch_render_k<32>(s, p, l, cam, rc, img, views, stride, st);
  return launch_render_k<64>(s, p, l, cam, rc, img, views, stride, st);
}

hipError_t launch_render(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l, const DevCam& cam,
                         const RasterConst& rc, const ngs_image& img, hipStream_t st) {
  return launch_render_views(s, p, l, cam, rc, img, 1, 0, st);
}

}  // namespace ngs
