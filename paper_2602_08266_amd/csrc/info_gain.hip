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
// wavefront forms its pixels' statistic contributions in registers and sums them over its
// 64 lanes with a recursive-halving reduce-scatter (64 statistics per round, 63 lane
// exchanges), after which lane s holds statistic s and adds it to the Gaussian's
// accumulator with one atomic. In both passes a wavefront only visits the batch entries whose
// conservative 3-sigma bounding box reaches its 16 x 4 pixel strip (a ballot mask); the
// skipped entries would fail the cut-off test at every one of its pixels.
#include "common.hpp"

namespace ngs {
namespace {

constexpr int kBatch = 32;

// Statistic s of a pixel is rv[i0] * rv[i1] * rv[i2] over the per-pixel record
// rv = (y[6], a, w_rgb[3], w_d, |w_rgb|^2, |w_o|^2, a T, 1, w_d^2), in the order of
// common.hpp: Y_rgb (upper 6x6), X_rgb (6x3), Y_d (upper 7x7 of e = (w_d y, a)), Y_o, m1.
struct StatDesc { unsigned char i0, i1, i2; };
struct StatTable { StatDesc d[kStatScalar]; };

constexpr StatTable make_stat_table() {
  StatTable t{};
  int s = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) t.d[s++] = {11, (unsigned char)i, (unsigned char)j};
  for (int i = 0; i < 6; ++i)
    for (int ch = 0; ch < 3; ++ch) t.d[s++] = {6, (unsigned char)i, (unsigned char)(7 + ch)};
  for (int i = 0; i < 7; ++i)
    for (int j = i; j < 7; ++j) {
      if (j < 6) t.d[s++] = {15, (unsigned char)i, (unsigned char)j};
      else if (i < 6) t.d[s++] = {10, (unsigned char)i, 6};
      else t.d[s++] = {6, 6, 14};
    }
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) t.d[s++] = {12, (unsigned char)i, (unsigned char)j};
  for (int i = 0; i < 6; ++i) t.d[s++] = {13, (unsigned char)i, 14};
  return t;
}
constexpr StatTable kStatTable = make_stat_table();
static_assert(kStatTable.d[kStatScalar - 1].i0 == 13 && kStatTable.d[kStatYd + 27].i2 == 14, "statistic table layout");

// Sums v over the 64 lanes of the wavefront and leaves entry l's total in lane l
// (recursive halving: at each step a lane keeps the half of its window selected by one bit
// of its lane id and adds the partner lane's copy of that half).
__device__ __forceinline__ float wave_reduce_scatter64(float (&v)[kWave], int lane) {
#pragma unroll
  for (int s = kWave / 2; s >= 1; s >>= 1) {
    const bool up = (lane & s) != 0;
#pragma unroll
    for (int i = 0; i < s; ++i) {
      const float send = up ? v[i] : v[i + s];
      const float keep = up ? v[i + s] : v[i];
      v[i] = keep + __shfl_xor(send, s);
    }
  }
  return v[0];
}

template <int KP>
struct IgShared {
  float mx[kBatch], my[kBatch], qa[kBatch], qb[kBatch], qc[kBatch], op[kBatch];
  float z[kBatch], r[kBatch], g[kBatch], b[kBatch], conf[kBatch], hx[kBatch], hy[kBatch];
  uint32_t gid[kBatch];
  float p[kBatch][KP];
  int flag;
};

// Whether batch entry l's ellipse can reach the wavefront's strip (entries past cnt: no).
template <class Sh>
__device__ __forceinline__ bool reaches(const Sh& S, int l, int cnt, float sx0, float sx1, float sy0, float sy1) {
  return l < cnt && S.mx[l] + S.hx[l] >= sx0 && S.mx[l] - S.hx[l] <= sx1 && S.my[l] + S.hy[l] >= sy0 &&
         S.my[l] - S.hy[l] <= sy1;
}

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
  // pixel-centre bounds of this wavefront's 16 x 4 strip
  const float sx0 = (float)(tx * kTile) + 0.5f, sx1 = sx0 + (float)(kTile - 1);
  const float sy0 = (float)(ty * kTile + wave * (kWave / kTile)) + 0.5f, sy1 = sy0 + (float)(kWave / kTile - 1);

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
      conic_extent(S.qa[j], S.qb[j], S.qc[j], rc.cutoff_q, &S.hx[j], &S.hy[j]);
    }
    __syncthreads();
    uint64_t live = __ballot(reaches(S, lane, cnt, sx0, sx1, sy0, sy1));
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
      conic_extent(S.qa[j], S.qb[j], S.qc[j], rc.cutoff_q, &S.hx[j], &S.hy[j]);
    }
    for (int idx = threadIdx.x; idx < cnt * KP; idx += kTilePix) {
      const int j = idx / KP, c = idx % KP;
      S.p[j][c] = (c < k) ? prob[(size_t)gids[lo + j] * k + c] : 0.f;
    }
    __syncthreads();
    uint64_t live = __ballot(reaches(S, lane, cnt, sx0, sx1, sy0, sy1));
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
        float rv[16] = {y0, y1, y2, y3, y4, y5, a, wr, wg, wb, wd, nrgb, no, a * Tg, 1.f, wd * wd};
        const float ao = a * om;
        const float zv[6] = {ao * y0, ao * y1, ao * y2, ao * y3, ao * y4, ao * y5};
        // Slot of this Gaussian in the per-view accumulator. A new slot is taken from the
        // counter, zeroed by the whole wavefront, and only then published in slot_of with a
        // compare-and-swap (a wavefront that loses the race leaves its zeroed slot unused,
        // marked by gid_of = -1); every later update of a published slot is an atomic add.
        const uint32_t gq = S.gid[j];
        int slot = -1, fresh = -1;
        if (lane == 0) {
          slot = __atomic_load_n(&slot_of[gq], __ATOMIC_RELAXED);
          if (slot < 0) {
            const int ns = atomicAdd(n_slots, 1);
            if (ns >= max_slots) atomicOr(overflow, 1); else fresh = ns;
          }
        }
        slot = __shfl(slot, 0);
        fresh = __shfl(fresh, 0);
        if (fresh >= 0) {
          for (int s = lane; s < stat_len(k); s += kWave) acc[(size_t)s * stride + fresh] = 0.f;
          __threadfence();
          __builtin_amdgcn_wave_barrier();
          if (lane == 0) {
            const int old = atomicCAS(&slot_of[gq], -1, fresh);
            gid_of[fresh] = (old == -1) ? (int)gq : -1;
            slot = (old == -1) ? fresh : old;
          }
          slot = __shfl(slot, 0);
        }
        if (slot >= 0) {
          // Sum this lane's contributions over the wavefront, 64 statistics at a time: the
          // padded statistic vector is [94 scalar statistics | Z_o as 6 x KP]; after the
          // reduce-scatter lane l holds entry 64 q + l of chunk q.
          constexpr int kLen = kStatScalar + 6 * KP;
#pragma unroll
          for (int q = 0; q < (kLen + kWave - 1) / kWave; ++q) {
            float v[kWave];
#pragma unroll
            for (int e = 0; e < kWave; ++e) {
              const int idx = q * kWave + e;
              if (idx < kStatScalar) {
                const StatDesc d = kStatTable.d[idx < kStatScalar ? idx : 0];
                v[e] = rv[d.i0] * rv[d.i1] * rv[d.i2];
              } else if (idx < kLen) {
                const int f = idx - kStatScalar;
                v[e] = zv[f / KP] * So[f % KP];
              } else {
                v[e] = 0.f;
              }
            }
            const float tot = wave_reduce_scatter64(v, lane);
            const int idx = q * kWave + lane;
            int dst = -1;
            if (idx < kStatScalar) {
              dst = idx;
            } else if (idx < kLen) {
              const int f = idx - kStatScalar, c = f % KP;
              if (c < k) dst = kStatScalar + (f / KP) * k + c;
            }
            if (dst >= 0 && tot != 0.f) atomicAdd(&acc[(size_t)dst * stride + slot], tot);
          }
        }
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
  hipError_t e = ig_reset(w, s.n, st);
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
