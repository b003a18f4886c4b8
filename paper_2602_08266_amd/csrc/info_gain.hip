// info_gain.hip -- per-tile accumulation of the screen-space information statistics.
//
// For every contributing (pixel, Gaussian) pair the Jacobian of each rendered channel w.r.t.
// the Gaussian's parameters factors as
//     d out_ch / d theta = w_ch * (d alpha / d theta) + direct feature terms,
//     w_ch = phi_ch T - S_ch / (1 - alpha),          S_ch = sum_{later j} phi_j,ch a_j,
// (compositing of Eq. 1; for the object vector of Eq. 2 the background channel also carries
// -T_final / (1 - alpha)). d alpha / d theta = P^T y with y = d alpha / d(m, Q, l) in screen
// space (6 numbers) and P = d(m, Q, l) / d theta per Gaussian. So the per-Gaussian block
// J^T J (Eq. 6, block diagonal) only needs per-pixel sums of products of y, a = alpha T and
// the w's: the 94 + 6k statistics listed in common.hpp. This kernel produces them; the
// FP64 chain rule through P, the blocks and the log-dets are in finalize.hip.
//
// One 256-lane workgroup per tile. Pass 1 walks front to back to find each pixel's final
// transmittance and last contributor. Pass 2 walks back to front from the tile's last
// contributor, recovering T before each Gaussian as T_after / (1 - alpha) and keeping the
// suffixes S in registers. For each Gaussian with a nonzero confidence weight, every
// wavefront writes one record per lane to LDS and reduces the statistics transposed: lane
// s sums statistic s over the 64 pixels (and lane k sums the k-th column of the 6 x k
// object term), then adds its result to the Gaussian's accumulator with one atomic.
#include "common.hpp"

namespace ngs {
namespace {

constexpr int kBatch = 32;
constexpr int kRecScalar = 22;  // y[6] a w_rgb[3] w_d |w_rgb|^2 |w_o|^2 aT 1 w_d^2 z[6]
constexpr int kChunk = 16;      // object-suffix channels transposed per round

// statistic s = rec[i0] * rec[i1] * rec[i2]
struct StatDesc { unsigned char i0, i1, i2; };
__constant__ StatDesc c_stats[kStatScalar];

template <int KP>
struct IgShared {
  float mx[kBatch], my[kBatch], qa[kBatch], qb[kBatch], qc[kBatch], op[kBatch];
  float z[kBatch], r[kBatch], g[kBatch], b[kBatch], conf[kBatch];
  uint32_t gid[kBatch];
  float p[kBatch][KP];
  static constexpr int kCh = KP < kChunk ? KP : kChunk;
  static constexpr int kRow = (kRecScalar + kCh) | 1;  // odd stride: conflict-free column reads
  float rec[kTilePix / kWave][kWave][kRow];
  int red_i[kTilePix / kWave];
  int red_new[kTilePix / kWave];
  int flag;
};

template <int KP>
__global__ __launch_bounds__(kTilePix) void k_ig_tile(
    int n, int k, const uint32_t* __restrict__ gids, const uint32_t* __restrict__ ranges, DevCam cam, RasterConst rc,
    const float* __restrict__ mean2d, const float* __restrict__ conic, const float* __restrict__ depth,
    const float* __restrict__ opacity, const float* __restrict__ rgb, const float* __restrict__ prob,
    const float* __restrict__ conf, int obj_eq2, float* __restrict__ acc, int32_t* __restrict__ slot_of,
    int32_t* __restrict__ gid_of, int32_t* __restrict__ n_slots, int32_t* __restrict__ overflow, int max_slots,
    int64_t* __restrict__ stats) {
  extern __shared__ unsigned char smem_raw[];
  IgShared<KP>& S = *reinterpret_cast<IgShared<KP>*>(smem_raw);
  const int ntiles = cam.tiles_x * cam.tiles_y;
  const int tile = blockIdx.x;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int px = tx * kTile + (threadIdx.x & (kTile - 1));
  const int py = ty * kTile + (threadIdx.x / kTile);
  const bool inside = px < cam.width && py < cam.height;
  const float fxp = (float)px + 0.5f, fyp = (float)py + 0.5f;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const uint32_t start = ranges[tile], end = ranges[ntiles + tile];
  const int stride = max_slots;

  // ---- pass 1: front to back, final transmittance and last contributor -----------------
  float T = 1.f;
  int last = -1, nc = 0;
  bool done = !inside;
  for (uint32_t b0 = start; b0 < end; b0 += kBatch) {
    if (__syncthreads_and(done)) break;
    const int cnt = (int)min((uint32_t)kBatch, end - b0);
    if ((int)threadIdx.x < cnt) {
      const uint32_t g = gids[b0 + threadIdx.x];
      const int j = threadIdx.x;
      S.mx[j] = mean2d[g]; S.my[j] = mean2d[n + g];
      S.qa[j] = conic[g]; S.qb[j] = conic[n + g]; S.qc[j] = conic[2 * n + g];
      S.op[j] = opacity[g];
    }
    __syncthreads();
    if (!done) {
      for (int j = 0; j < cnt; ++j) {
        const float dx = fxp - S.mx[j], dy = fyp - S.my[j];
        const float q = conic_q(S.qa[j], S.qb[j], S.qc[j], dx, dy);
        if (q > rc.cutoff_q) continue;
        const float alpha = fminf(rc.alpha_max, gauss_alpha(S.op[j], q));
        if (alpha < rc.alpha_min) continue;
        const float Tn = transmit(T, alpha);
        if (Tn < rc.t_min) { done = true; break; }
        T = Tn;
        last = (int)(b0 + j);
        ++nc;
      }
    }
  }
  // tile extent of pass 2 and whether any walked Gaussian carries weight
  if (threadIdx.x == 0) S.flag = -1;
  __syncthreads();
  if (last >= 0) atomicMax(&S.flag, last);
  __syncthreads();
  const int tile_last = S.flag;
  if (stats) {
    // contributing (pixel, Gaussian) pairs P
    int tot = nc;
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
    if (lane == 0 && tot) atomicAdd((unsigned long long*)&stats[3], (unsigned long long)tot);
    if (threadIdx.x == 0 && tile_last >= 0)
      atomicAdd((unsigned long long*)&stats[4], (unsigned long long)(tile_last - (int)start + 1));
  }
  if (tile_last < 0) return;
  __syncthreads();
  if (threadIdx.x == 0) S.flag = 0;
  __syncthreads();
  for (int i = (int)start + threadIdx.x; i <= tile_last; i += kTilePix)
    if (conf[gids[i]] > 0.f) S.flag = 1;
  __syncthreads();
  if (S.flag == 0) return;

  // ---- pass 2: back to front ------------------------------------------------------------
  const float t_final = T;
  float Tc = T;
  float Sr = 0.f, Sg = 0.f, Sb = 0.f, Sd = 0.f;
  float So[KP];
#pragma unroll
  for (int c = 0; c < KP; ++c) So[c] = 0.f;
  if (obj_eq2) So[0] = t_final;  // S~ = S_o + T_final e_0
  float* rec = &S.rec[wave][lane][0];
  for (int hi = tile_last + 1; hi > (int)start; hi -= kBatch) {
    const int lo = max((int)start, hi - kBatch);
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
      S.conf[j] = conf[g];
    }
    for (int idx = threadIdx.x; idx < cnt * KP; idx += kTilePix) {
      const int j = idx / KP, c = idx % KP;
      S.p[j][c] = (c < k) ? prob[(size_t)gids[lo + j] * k + c] : 0.f;
    }
    __syncthreads();
    for (int j = cnt - 1; j >= 0; --j) {
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
      float a = 0.f, Tg = 0.f, om = 0.f;
      if (contrib) {
        om = 1.f / (1.f - alpha);
        Tg = Tc * om;
        a = alpha * Tg;
      }
      const float cw = S.conf[j];
      if (cw > 0.f && __any(contrib)) {
        // record of this lane's pixel (zeros when it does not contribute)
        float y0 = 0.f, y1 = 0.f, y2 = 0.f, y3 = 0.f, y4 = 0.f, y5 = 0.f;
        float wr = 0.f, wg = 0.f, wb = 0.f, wd = 0.f, nrgb = 0.f, no = 0.f;
        if (contrib) {
          if (raw < rc.alpha_max) {
            y0 = alpha * (S.qa[j] * dx + S.qb[j] * dy);
            y1 = alpha * (S.qb[j] * dx + S.qc[j] * dy);
            y2 = -0.5f * alpha * dx * dx;
            y3 = -alpha * dx * dy;
            y4 = -0.5f * alpha * dy * dy;
            y5 = alpha * (1.f - S.op[j]);
          }
          wr = S.r[j] * Tg - Sr * om;
          wg = S.g[j] * Tg - Sg * om;
          wb = S.b[j] * Tg - Sb * om;
          wd = S.z[j] * Tg - Sd * om;
          nrgb = wr * wr + wg * wg + wb * wb;
#pragma unroll
          for (int c = 0; c < KP; ++c) {
            const float w = S.p[j][c] * Tg - So[c] * om;
            no += w * w;
          }
        }
        const float ao = a * om;
        rec[0] = y0; rec[1] = y1; rec[2] = y2; rec[3] = y3; rec[4] = y4; rec[5] = y5;
        rec[6] = a; rec[7] = wr; rec[8] = wg; rec[9] = wb; rec[10] = wd; rec[11] = nrgb; rec[12] = no;
        rec[13] = a * Tg; rec[14] = 1.f; rec[15] = wd * wd;
        rec[16] = ao * y0; rec[17] = ao * y1; rec[18] = ao * y2; rec[19] = ao * y3; rec[20] = ao * y4;
        rec[21] = ao * y5;
        // Slot of this Gaussian in the per-view accumulator. A new slot is taken from the
        // counter, zeroed by the whole wavefront, and only then published in slot_of with a
        // compare-and-swap (a wavefront that loses the race leaves its zeroed slot unused,
        // marked by gid_of = -1); every later update of a published slot is an atomic add.
        const uint32_t gq = S.gid[j];
        if (lane == 0) {
          int s = __atomic_load_n(&slot_of[gq], __ATOMIC_RELAXED);
          int fresh = -1;
          if (s < 0) {
            const int ns = atomicAdd(n_slots, 1);
            if (ns >= max_slots) atomicOr(overflow, 1); else fresh = ns;
          }
          S.red_i[wave] = s;
          S.red_new[wave] = fresh;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int fresh = S.red_new[wave];
        if (fresh >= 0) {
          for (int s = lane; s < stat_len(k); s += kWave) acc[(size_t)s * stride + fresh] = 0.f;
          __threadfence();
          __builtin_amdgcn_wave_barrier();
          if (lane == 0) {
            const int old = atomicCAS(&slot_of[gq], -1, fresh);
            gid_of[fresh] = (old == -1) ? (int)gq : -1;
            S.red_i[wave] = (old == -1) ? fresh : old;
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        const int slot = S.red_i[wave];
        if (slot >= 0) {
          const float* rows = &S.rec[wave][0][0];
          constexpr int R = IgShared<KP>::kRow;
          constexpr int CH = IgShared<KP>::kCh;
          // scalar statistics: lane s handles s and s + 64
          for (int s = lane; s < kStatScalar; s += kWave) {
            const StatDesc d = c_stats[s];
            float v = 0.f;
            for (int p = 0; p < kWave; ++p) {
              const float* rp = rows + p * R;
              v += rp[d.i0] * rp[d.i1] * rp[d.i2];
            }
            if (v != 0.f) atomicAdd(&acc[(size_t)s * stride + slot], v);
          }
          // object term Z_o[i][c] = sum_p z_i S~_c, CH channels per round; lanes form
          // groups of CH channels that split the 64 pixels, then combine by shuffles.
          constexpr int G = kWave / CH;
          const int cl = lane % CH, grp = lane / CH;
#pragma unroll
          for (int c0 = 0; c0 < KP; c0 += CH) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
            for (int c = 0; c < CH; ++c) rec[kRecScalar + c] = contrib ? So[c0 + c] : 0.f;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            float zz[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            for (int p = grp; p < kWave; p += G) {
              const float* rp = rows + p * R;
              const float sv = rp[kRecScalar + cl];
#pragma unroll
              for (int i = 0; i < 6; ++i) zz[i] += rp[16 + i] * sv;
            }
#pragma unroll
            for (int off = CH; off < kWave; off <<= 1)
#pragma unroll
              for (int i = 0; i < 6; ++i) zz[i] += __shfl_xor(zz[i], off);
            const int c = c0 + cl;
            if (grp == 0 && c < k)
#pragma unroll
              for (int i = 0; i < 6; ++i)
                if (zz[i] != 0.f) atomicAdd(&acc[(size_t)(kStatScalar + i * k + c) * stride + slot], zz[i]);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
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

__global__ void k_ig_clear(int32_t* n_slots, int32_t* overflow) {
  *n_slots = 0;
  *overflow = 0;
}

template <int KP>
hipError_t launch_ig_k(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l, const DevCam& cam,
                       const RasterConst& rc, const ngs_ig_params& ig, const IgWs& w, int64_t* stats, hipStream_t st) {
  const int ntiles = cam.tiles_x * cam.tiles_y;
  const size_t shm = sizeof(IgShared<KP>);
  ProfScope ps(kProfIgTiles, st);
  hipLaunchKernelGGL(k_ig_tile<KP>, dim3(ntiles), dim3(kTilePix), shm, st, s.n, s.k, l.gids, l.ranges, cam, rc,
                     p.mean2d, p.conic, p.depth, s.opacity, s.rgb, s.prob, s.conf, ig.obj_eq2, w.acc, w.slot_of,
                     w.gid_of, w.n_slots, w.overflow, (int)w.max_slots, stats);
  return hipGetLastError();
}

bool g_stats_uploaded = false;

hipError_t upload_stat_table() {
  if (g_stats_uploaded) return hipSuccess;
  StatDesc t[kStatScalar];
  int s = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) t[s++] = {11, (unsigned char)i, (unsigned char)j};          // Y_rgb
  for (int i = 0; i < 6; ++i)
    for (int ch = 0; ch < 3; ++ch) t[s++] = {6, (unsigned char)i, (unsigned char)(7 + ch)};  // X_rgb
  for (int i = 0; i < 7; ++i)
    for (int j = i; j < 7; ++j) {                                                            // Y_d
      if (j < 6) t[s++] = {15, (unsigned char)i, (unsigned char)j};
      else if (i < 6) t[s++] = {10, (unsigned char)i, 6};
      else t[s++] = {6, 6, 14};
    }
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) t[s++] = {12, (unsigned char)i, (unsigned char)j};          // Y_o
  for (int i = 0; i < 6; ++i) t[s++] = {13, (unsigned char)i, 14};                          // m1
  if (s != kStatScalar) return hipErrorInvalidValue;
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_stats), t, sizeof(t));
  if (e == hipSuccess) g_stats_uploaded = true;
  return e;
}

}  // namespace

size_t ig_ws_bytes(int64_t n, int64_t k, int64_t max_slots) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  return al((size_t)stat_len((int)k) * (size_t)max_slots * 4) + al((size_t)std::max<int64_t>(n, 1) * 4) +
         al((size_t)max_slots * 4) + al(8);
}

IgWs ig_ws_carve(void* ws, int64_t n, int64_t k, int64_t max_slots) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  char* p = static_cast<char*>(ws);
  IgWs w;
  w.acc = (float*)p; p += al((size_t)stat_len((int)k) * (size_t)max_slots * 4);
  w.slot_of = (int32_t*)p; p += al((size_t)std::max<int64_t>(n, 1) * 4);
  w.gid_of = (int32_t*)p; p += al((size_t)max_slots * 4);
  w.n_slots = (int32_t*)p;
  w.overflow = w.n_slots + 1;
  w.max_slots = max_slots;
  return w;
}

// Per-view reset: no Gaussian holds a slot. Accumulator slots are zeroed when taken.
hipError_t ig_reset(const IgWs& w, int n, hipStream_t st) {
  return launch_fill_i32(w.slot_of, -1, (size_t)std::max(n, 1), st);
}

hipError_t launch_ig_tiles(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l, const DevCam& cam,
                           const RasterConst& rc, const ngs_ig_params& ig, const IgWs& w, int64_t* stats,
                           hipStream_t st) {
  hipError_t e = upload_stat_table();
  if (e != hipSuccess) return e;
  e = ig_reset(w, s.n, st);
  if (e != hipSuccess) return e;
  {
    ProfScope ps(kProfFill, st);
    hipLaunchKernelGGL(k_ig_clear, dim3(1), dim3(1), 0, st, w.n_slots, w.overflow);
  }
  if (s.k <= 4) return launch_ig_k<4>(s, p, l, cam, rc, ig, w, stats, st);
  if (s.k <= 8) return launch_ig_k<8>(s, p, l, cam, rc, ig, w, stats, st);
  if (s.k <= 16) return launch_ig_k<16>(s, p, l, cam, rc, ig, w, stats, st);
  if (s.k <= 32) return launch_ig_k<32>(s, p, l, cam, rc, ig, w, stats, st);
  return launch_ig_k<64>(s, p, l, cam, rc, ig, w, stats, st);
}

}  // namespace ngs
