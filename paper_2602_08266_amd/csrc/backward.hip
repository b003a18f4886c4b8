// backward.hip -- backward rasterizer: gradients of a loss w.r.t. the Gaussian parameters,
// given the loss gradients w.r.t. the rendered colour, depth and object images (scene
// refinement, Sec. III-A.2; compositing of Eq. 1-2).
//
// The same factorisation as the information gain: for a contributing (pixel, Gaussian) pair,
// d out_ch / d theta = w_ch * d alpha / d theta + direct terms, with
// w_ch = phi_ch T - S_ch / (1 - alpha) (S_ch: suffix of later contributors; for the object
// vector O of Eq. 2 channel 0 also carries -T_final / (1 - alpha)) and d alpha / d theta =
// P^T y, y = d alpha / d(m_x, m_y, Q_xx, Q_xy, Q_yy, l). So per pixel
//   dL / d alpha = sum_ch g_ch w_ch,
// and per Gaussian, summed over its pixels:
//   screen gradient  G_u = sum (dL / d alpha) y            (6)
//   depth feature    G_z = sum a g_D                        (D = sum Z a: Z also moves with mu)
//   colour           G_c = sum a g_rgb                      (3)
//   probabilities    G_p = sum a g_O                        (k; through the softmax below)
// with a = alpha T. k_bwd_tile walks every tile back to front and accumulates (G_u, G_z, G_c,
// G_p) per Gaussian; k_bwd_params applies the FP64 chain rule of the projection (P, dZ/dmu)
// and the softmax Jacobian: dL/d o = p * (G_p - p . G_p).
#include "chain.hpp"
#include "common.hpp"

namespace ngs {
namespace {

constexpr int kBwBatch = 32;
constexpr int kBwChunk = 16;   // packed rows per reduction round
constexpr int kBwScal = 12;    // G_u 6, G_z, G_c 3, padding 2
constexpr int kSgHead = 16;    // screen-gradient row: [G_u 6 | G_z | G_c 3 | pad 6 | G_p k]

inline __host__ __device__ int sg_stride(int k) { return kSgHead + k; }

template <int KP>
struct BwShared {
  float mx[kBwBatch], my[kBwBatch], qa[kBwBatch], qb[kBwBatch], qc[kBwBatch], op[kBwBatch];
  float z[kBwBatch], r[kBwBatch], g[kBwBatch], b[kBwBatch], hx[kBwBatch], hy[kBwBatch];
  uint32_t gid[kBwBatch];
  float p[kBwBatch][KP];
  float srow[kTilePix / kWave][kBwChunk][kBwScal];
  float prow[kTilePix / kWave][kBwChunk][KP + 4];
  int flag;
};

template <class Sh>
__device__ __forceinline__ bool bw_reaches(const Sh& S, int l, int cnt, float sx0, float sx1, float sy0, float sy1) {
  return l < cnt && S.mx[l] + S.hx[l] >= sx0 && S.mx[l] - S.hx[l] <= sx1 && S.my[l] + S.hy[l] >= sy0 &&
         S.my[l] - S.hy[l] <= sy1;
}

template <int KP>
__global__ __launch_bounds__(kTilePix) void k_bwd_tile(
    int n, int k, const uint32_t* __restrict__ gids, const uint32_t* __restrict__ ranges, DevCam cam, RasterConst rc,
    const float* __restrict__ mean2d, const float* __restrict__ conic, const float* __restrict__ depth,
    const float* __restrict__ opacity, const float* __restrict__ rgb, const float* __restrict__ prob, int obj_eq2,
    const float* __restrict__ g_rgb, const float* __restrict__ g_depth, const float* __restrict__ g_obj,
    float* __restrict__ sg) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  BwShared<KP>& S = *reinterpret_cast<BwShared<KP>*>(smem_raw);
  const int ntiles = cam.tiles_x * cam.tiles_y;
  const int tile = blockIdx.x;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int px = tx * kTile + (threadIdx.x & (kTile - 1));
  const int py = ty * kTile + (threadIdx.x / kTile);
  const bool inside = px < cam.width && py < cam.height;
  const float fxp = (float)px + 0.5f, fyp = (float)py + 0.5f;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const uint32_t start = ranges[tile], end = ranges[ntiles + tile];
  const int stride = sg_stride(k);
  const float sx0 = (float)(tx * kTile) + 0.5f, sx1 = sx0 + (float)(kTile - 1);
  const float sy0 = (float)(ty * kTile + wave * (kWave / kTile)) + 0.5f, sy1 = sy0 + (float)(kWave / kTile - 1);

  // ---- pass 1: front to back, final transmittance and last contributor -----------------
  float T = 1.f;
  int last = -1;
  bool done = !inside;
  for (uint32_t b0 = start; b0 < end; b0 += kBwBatch) {
    if (__syncthreads_and(done)) break;
    const int cnt = (int)min((uint32_t)kBwBatch, end - b0);
    if ((int)threadIdx.x < cnt) {
      const uint32_t g = gids[b0 + threadIdx.x];
      const int j = threadIdx.x;
      S.mx[j] = mean2d[g]; S.my[j] = mean2d[n + g];
      S.qa[j] = conic[g]; S.qb[j] = conic[n + g]; S.qc[j] = conic[2 * n + g];
      S.op[j] = opacity[g];
      conic_extent(S.qa[j], S.qb[j], S.qc[j], rc.cutoff_q, &S.hx[j], &S.hy[j]);
    }
    __syncthreads();
    uint64_t live = __ballot(bw_reaches(S, lane, cnt, sx0, sx1, sy0, sy1));
    if (!done) {
      while (live) {
        const int j = __ffsll((unsigned long long)live) - 1;
        live &= live - 1;
        const float dx = fxp - S.mx[j], dy = fyp - S.my[j];
        const float q = conic_q(S.qa[j], S.qb[j], S.qc[j], dx, dy);
        if (q > rc.cutoff_q) continue;
        const float alpha = fminf(rc.alpha_max, gauss_alpha(S.op[j], q));
        if (alpha < rc.alpha_min) continue;
        const float Tn = transmit(T, alpha);
        if (Tn < rc.t_min) { done = true; break; }
        T = Tn;
        last = (int)(b0 + j);
      }
    }
  }
  if (threadIdx.x == 0) S.flag = -1;
  __syncthreads();
  if (last >= 0) atomicMax(&S.flag, last);
  __syncthreads();
  const int tile_last = S.flag;
  if (tile_last < 0) return;

  // this pixel's loss gradients (zero outside the image)
  const size_t HW = (size_t)cam.width * cam.height;
  const size_t pix = inside ? (size_t)py * cam.width + px : 0;
  float gc[3] = {0.f, 0.f, 0.f}, gd = 0.f, go[KP];
#pragma unroll
  for (int c = 0; c < KP; ++c) go[c] = 0.f;
  if (inside) {
    if (g_rgb)
      for (int ch = 0; ch < 3; ++ch) gc[ch] = g_rgb[ch * HW + pix];
    if (g_depth) gd = g_depth[pix];
    if (g_obj) {
#pragma unroll
      for (int c = 0; c < KP; ++c) go[c] = c < k ? g_obj[c * HW + pix] : 0.f;
    }
  }

  // ---- pass 2: back to front ------------------------------------------------------------
  const float t_final = T;
  float Tc = T;
  float Sr = 0.f, Sg = 0.f, Sb = 0.f, Sd = 0.f;
  float So[KP];
#pragma unroll
  for (int c = 0; c < KP; ++c) So[c] = 0.f;
  if (obj_eq2) So[0] = t_final;  // S~ = S_o + T_final e_0
  for (int hi = tile_last + 1; hi > (int)start; hi -= kBwBatch) {
    const int lo = max((int)start, hi - kBwBatch);
    const int cnt = hi - lo;
    __syncthreads();
    if ((int)threadIdx.x < cnt) {
      const int j = threadIdx.x;
      const uint32_t g = gids[lo + j];
      S.gid[j] = g;
      S.mx[j] = mean2d[g]; S.my[j] = mean2d[n + g];
      S.qa[j] = conic[g]; S.qb[j] = conic[n + g]; S.qc[j] = conic[2 * n + g];
      S.op[j] = opacity[g]; S.z[j] = depth[g];
      S.r[j] = rgb[g]; S.g[j] = rgb[n + g]; S.b[j] = rgb[2 * n + g];
      conic_extent(S.qa[j], S.qb[j], S.qc[j], rc.cutoff_q, &S.hx[j], &S.hy[j]);
    }
    for (int idx = threadIdx.x; idx < cnt * KP; idx += kTilePix) {
      const int j = idx / KP, c = idx % KP;
      S.p[j][c] = (c < k) ? prob[(size_t)gids[lo + j] * k + c] : 0.f;
    }
    __syncthreads();
    uint64_t live = __ballot(bw_reaches(S, lane, cnt, sx0, sx1, sy0, sy1));
    while (live) {
      const int j = 63 - __clzll((long long)live);
      live &= ~(1ull << j);
      const int li = lo + j;
      bool contrib = false;
      float alpha = 0.f, dx = 0.f, dy = 0.f, raw = 0.f;
      if (li <= last) {
        dx = fxp - S.mx[j];
        dy = fyp - S.my[j];
        const float q = conic_q(S.qa[j], S.qb[j], S.qc[j], dx, dy);
        if (q <= rc.cutoff_q) {
          raw = gauss_alpha(S.op[j], q);
          alpha = fminf(rc.alpha_max, raw);
          contrib = alpha >= rc.alpha_min;
        }
      }
      const uint64_t cmask = __ballot(contrib);
      if (!cmask) continue;
      float a = 0.f, Tg = 0.f, om = 0.f;
      float row[kBwScal];
#pragma unroll
      for (int e = 0; e < kBwScal; ++e) row[e] = 0.f;
      if (contrib) {
        om = 1.f / (1.f - alpha);
        Tg = Tc * om;
        a = alpha * Tg;
        // dL / d alpha over every channel
        float dla = gc[0] * (S.r[j] * Tg - Sr * om) + gc[1] * (S.g[j] * Tg - Sg * om) +
                    gc[2] * (S.b[j] * Tg - Sb * om) + gd * (S.z[j] * Tg - Sd * om);
#pragma unroll
        for (int c = 0; c < KP; ++c) dla += go[c] * (S.p[j][c] * Tg - So[c] * om);
        if (raw < rc.alpha_max) {
          row[0] = dla * alpha * (S.qa[j] * dx + S.qb[j] * dy);
          row[1] = dla * alpha * (S.qb[j] * dx + S.qc[j] * dy);
          row[2] = dla * (-0.5f * alpha * dx * dx);
          row[3] = dla * (-alpha * dx * dy);
          row[4] = dla * (-0.5f * alpha * dy * dy);
          row[5] = dla * alpha * (1.f - S.op[j]);
        }
        row[6] = a * gd;
        row[7] = a * gc[0]; row[8] = a * gc[1]; row[9] = a * gc[2];
      }
      // Sum the contributing lanes' rows (and a * g_O) over the wavefront: rows packed by
      // rank into LDS, 16 at a time; lane e < 10 sums scalar column e, lane c < KP sums
      // object column c; then one atomic per column into the Gaussian's row.
      const int cnt_c = __popcll(cmask);
      const int rank = __popcll(cmask & ((1ull << lane) - 1ull));
      float (*sr)[kBwScal] = S.srow[wave];
      float (*pr)[KP + 4] = S.prow[wave];
      float accS = 0.f, accP = 0.f;
      for (int c0 = 0; c0 < cnt_c; c0 += kBwChunk) {
        if (contrib && rank >= c0 && rank < c0 + kBwChunk) {
          float* d = sr[rank - c0];
#pragma unroll
          for (int e = 0; e < kBwScal; e += 4) *reinterpret_cast<float4*>(d + e) = make_float4(row[e], row[e + 1], row[e + 2], row[e + 3]);
          float* dp = pr[rank - c0];
#pragma unroll
          for (int c = 0; c < KP; c += 4)
            *reinterpret_cast<float4*>(dp + c) = make_float4(a * go[c], a * go[c + 1], a * go[c + 2], a * go[c + 3]);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        const int m = min(kBwChunk, cnt_c - c0);
        for (int rr = 0; rr < m; ++rr) {
          if (lane < 10) accS += sr[rr][lane];
          if (lane < KP) accP += pr[rr][lane];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      }
      float* dst = sg + (size_t)S.gid[j] * stride;
      if (lane < 10 && accS != 0.f) atomicAdd(dst + lane, accS);
      if (lane < k && accP != 0.f) atomicAdd(dst + kSgHead + lane, accP);
      if (contrib) {
        Sr += S.r[j] * a; Sg += S.g[j] * a; Sb += S.b[j] * a;
        Sd += S.z[j] * a;
#pragma unroll
        for (int c = 0; c < KP; ++c) So[c] += S.p[j][c] * a;
        Tc = Tg;
      }
    }
  }
}

// Parameter gradients of every Gaussian from its screen gradient (FP64 chain rule).
__global__ __launch_bounds__(256) void k_bwd_params(
    int n, int k, const float* __restrict__ mean, const float* __restrict__ log_scale, const float* __restrict__ rot,
    const float* __restrict__ prob, const uint32_t* __restrict__ count, DevCam cam, double eps2d,
    const float* __restrict__ sg, ngs_scene_grad out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const float* row = sg + (size_t)g * sg_stride(k);
  double gu[6], gz = 0.0;
  bool any = false;
  for (int a = 0; a < 6; ++a) { gu[a] = row[a]; any |= row[a] != 0.f; }
  gz = row[6];
  any |= row[6] != 0.f;
  double dth[kNGeo];
  for (int j = 0; j < kNGeo; ++j) dth[j] = 0.0;
  if (count[g] > 0u && any) {
    double P[7][kNGeo];
    chain_rule(mean, log_scale, rot, n, g, cam, eps2d, P);
    for (int j = 0; j < kNGeo; ++j) {
      double v = gz * P[6][j];
      for (int a = 0; a < 6; ++a) v += gu[a] * P[a][j];
      dth[j] = v;
    }
  }
  for (int i = 0; i < 3; ++i) out.mean[(size_t)i * n + g] = (float)dth[i];
  for (int i = 0; i < 3; ++i) out.log_scale[(size_t)i * n + g] = (float)dth[3 + i];
  for (int i = 0; i < 4; ++i) out.rot[(size_t)i * n + g] = (float)dth[6 + i];
  out.opacity_logit[g] = (float)dth[10];
  for (int ch = 0; ch < 3; ++ch) out.rgb[(size_t)ch * n + g] = row[7 + ch];
  // softmax: d L / d o_j = p_j (G_p,j - sum_m p_m G_p,m)
  const float* pg = prob + (size_t)g * k;
  double dot = 0.0;
  for (int m = 0; m < k; ++m) dot += (double)pg[m] * row[kSgHead + m];
  for (int j = 0; j < k; ++j) out.obj_logit[(size_t)j * n + g] = (float)((double)pg[j] * ((double)row[kSgHead + j] - dot));
}

__global__ void k_bwd_zero(float4* __restrict__ v, size_t n4) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (size_t)gridDim.x * blockDim.x)
    v[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int KP>
hipError_t launch_bwd_k(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l, const DevCam& cam,
                        const RasterConst& rc, int obj_eq2, const ngs_image_grad& gi, float* sg, hipStream_t st) {
  const int ntiles = cam.tiles_x * cam.tiles_y;
  const size_t shm = sizeof(BwShared<KP>);
  static_assert(sizeof(BwShared<KP>) <= 65536, "backward kernel LDS");
  ProfScope ps(kProfBwdTiles, st);
  hipLaunchKernelGGL((k_bwd_tile<KP>), dim3(ntiles), dim3(kTilePix), shm, st, s.n, s.k, l.gids, l.ranges, cam, rc,
                     p.mean2d, p.conic, p.depth, s.opacity, s.rgb, s.prob, obj_eq2, gi.rgb, gi.depth, gi.obj, sg);
  return hipGetLastError();
}

}  // namespace

size_t bwd_ws_bytes(int64_t n, int64_t k) {
  return ((size_t)std::max<int64_t>(n, 1) * (size_t)sg_stride((int)k) * 4 + 255) / 256 * 256;
}

hipError_t launch_render_backward(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l,
                                  const DevCam& cam, const ngs_raster_params& rp, int obj_eq2,
                                  const ngs_image_grad& gi, const ngs_scene_grad& out, void* ws, hipStream_t st) {
  float* sg = static_cast<float*>(ws);
  const size_t n4 = (size_t)std::max(s.n, 1) * sg_stride(s.k) / 4;
  {
    ProfScope ps(kProfFill, st);
    hipLaunchKernelGGL(k_bwd_zero, dim3(1024), dim3(256), 0, st, reinterpret_cast<float4*>(sg), n4);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const RasterConst rc = make_raster(rp);
  if (s.k <= 4) e = launch_bwd_k<4>(s, p, l, cam, rc, obj_eq2, gi, sg, st);
  else if (s.k <= 8) e = launch_bwd_k<8>(s, p, l, cam, rc, obj_eq2, gi, sg, st);
  else if (s.k <= 16) e = launch_bwd_k<16>(s, p, l, cam, rc, obj_eq2, gi, sg, st);
  else if (s.k <= 32) e = launch_bwd_k<32>(s, p, l, cam, rc, obj_eq2, gi, sg, st);
  else e = launch_bwd_k<64>(s, p, l, cam, rc, obj_eq2, gi, sg, st);
  if (e != hipSuccess) return e;
  if (s.n > 0) {
    ProfScope ps(kProfBwdParams, st);
    hipLaunchKernelGGL(k_bwd_params, dim3((s.n + 255) / 256), dim3(256), 0, st, s.n, s.k, s.mean, s.log_scale, s.rot,
                       s.prob, p.count, cam, (double)rp.eps2d, sg, out);
  }
  return hipGetLastError();
}

}  // namespace ngs
