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
// The walk runs in three launches per view:
//   1. k_ig_front, one 256-lane workgroup per tile, one lane per pixel: the front-to-back pass
//      that gives each pixel its final transmittance and its last contributor (stored per
//      pixel); the first contribution of a Gaussian with a nonzero confidence weight claims
//      its accumulator slot (U of them; every other Gaussian keeps slot -1 and is never
//      reduced; the finalisation sets the claimed ones back to -1 for the next view);
//   2. k_ig_zero: the claimed slots' statistics zeroed;
//   3. k_ig_back, one workgroup per tile with one, two or four lanes per pixel: the
//      back-to-front pass from the tile's last contributor, recovering T before each Gaussian
//      as T_after / (1 - alpha) and keeping the suffixes S in registers. For each slotted
//      Gaussian, the wavefront's contributing lanes write their per-pixel records (and object
//      suffixes) to LDS rows, packed by rank, 16 rows at a time; then every lane owns
//      statistics (one or two scalar ones and the six Z_o entries of one object channel) and
//      sums them over the packed rows only, so the cost follows the number of contributing
//      pixels, not the 64 lanes. The sums go to the slot with atomic adds on contiguous
//      addresses.
// In both passes a wavefront only visits the batch entries whose conservative 3-sigma
// bounding box reaches its 16 x 4 pixel strip (a ballot mask); the skipped entries would fail
// the cut-off test at every one of its pixels. With a target object (Eq. 12) a pre-pass marks
// the tiles that the rect of a weighted Gaussian reaches, and both passes leave the others.
#include "common.hpp"

namespace ngs {
namespace {

// Entries staged per back-pass batch: 64 with one lane per pixel (fewer batch barriers), 32 in
// the wider workgroups, whose LDS holds more record rows.
template <int LPP> constexpr int batch_entries() { return LPP == 1 ? 64 : 32; }

// Per-pixel record of a contributing (pixel, Gaussian) pair, laid out so that every scalar
// statistic of common.hpp is the product of two of its entries:
//   [0, 6) y   [6, 12) |w_rgb|^2 y   [12, 18) |w_o|^2 y   [18, 24) w_d^2 y
//   [24, 30) a / (1 - alpha) y  (Z_o's left factor)
//   30 a w_r, 31 a w_g, 32 a w_b, 33 a w_d, 34 a T, 35 a
// y = d alpha / d(m_x, m_y, Q_xx, Q_xy, Q_yy, l), a = alpha T, w = d out / d alpha.
constexpr int kRec = 36;  // 36 floats apart: the 16 rows of a chunk start on distinct 4-bank groups
constexpr int kRecZ = 24, kRecAW = 30, kRecAT = 34, kRecA = 35;

struct StatPair { unsigned char u, v; };
struct StatTable { StatPair d[kStatScalar]; };

constexpr StatTable make_stat_table() {
  StatTable t{};
  int s = 0;
  for (int i = 0; i < 6; ++i)  // Y_rgb
    for (int j = i; j < 6; ++j) t.d[s++] = {(unsigned char)(6 + i), (unsigned char)j};
  for (int i = 0; i < 6; ++i)  // X_rgb
    for (int ch = 0; ch < 3; ++ch) t.d[s++] = {(unsigned char)i, (unsigned char)(kRecAW + ch)};
  for (int i = 0; i < 7; ++i)  // Y_d over e = (w_d y, a)
    for (int j = i; j < 7; ++j) {
      if (j < 6) t.d[s++] = {(unsigned char)(18 + i), (unsigned char)j};
      else if (i < 6) t.d[s++] = {(unsigned char)i, (unsigned char)(kRecAW + 3)};
      else t.d[s++] = {(unsigned char)kRecA, (unsigned char)kRecA};
    }
  for (int i = 0; i < 6; ++i)  // Y_o
    for (int j = i; j < 6; ++j) t.d[s++] = {(unsigned char)(12 + i), (unsigned char)j};
  for (int i = 0; i < 6; ++i) t.d[s++] = {(unsigned char)i, (unsigned char)kRecAT};  // m1
  return t;
}
constexpr StatTable kStatTable = make_stat_table();
static_assert(kStatTable.d[kStatM1].v == kRecAT && kStatTable.d[kStatYd + 27].u == kRecA, "statistic table layout");

__constant__ StatTable c_stats = make_stat_table();

// Packed rows per reduction round: 16, or 8 when four lanes share a pixel (16 pixels per
// wavefront) so that the rows of all 16 wavefronts fit in LDS.
template <int LPP> constexpr int chunk_rows() { return LPP == 4 ? 8 : 16; }

// Adds R packed rows (R a multiple of 4) into this lane's statistics: the scalar statistics
// (u_a, v_a) and (u_b, v_b), and Z_o for channel zc over the rows of its pixel group. Rows past
// the contributing lanes hold zero records, so no row needs masking.
template <int KP>
__device__ __forceinline__ void reduce_rows(int R, const float (*rec)[kRec], const float (*sov)[KP + 4], int ua,
                                            int va, int ub, int vb, int grp, int zc, float& accA, float& accB,
                                            float (&z)[6]) {
  constexpr int kGroups = kWave / KP;
  constexpr int kStep = 4;  // rows per iteration: enough loads in flight, few registers
#pragma unroll 1
  for (int r0 = 0; r0 < R; r0 += kStep) {
#pragma unroll
    for (int r = r0; r < r0 + kStep; ++r) {
      accA += rec[r][ua] * rec[r][va];
      accB += rec[r][ub] * rec[r][vb];
    }
  }
  const int rows_per_group = (R + kGroups - 1) / kGroups;
#pragma unroll 1
  for (int t0 = 0; t0 < rows_per_group; t0 += kStep) {
#pragma unroll
    for (int t = t0; t < t0 + kStep; ++t) {
      const int r = t * kGroups + grp;
      if (kGroups > 1 && t * kGroups >= R) break;
      const int rr = r < R ? r : R - 1;
      const float4 u = *reinterpret_cast<const float4*>(&rec[rr][kRecZ]);
      const float2 v = *reinterpret_cast<const float2*>(&rec[rr][kRecZ + 4]);
      const float sv = r < R ? sov[rr][zc] : 0.f;
      z[0] += u.x * sv; z[1] += u.y * sv; z[2] += u.z * sv; z[3] += u.w * sv;
      z[4] += v.x * sv; z[5] += v.y * sv;
    }
  }
}

template <int KP, int LPP>
struct IgShared {
  static constexpr int kB = batch_entries<LPP>();
  float mx[kB], my[kB], qa[kB], qb[kB], qc[kB], op[kB];
  float z[kB], r[kB], g[kB], b[kB], hx[kB], hy[kB];
  int32_t slot[kB];
  float p[kB][KP];
  float rec[kTilePix * LPP / kWave][chunk_rows<LPP>()][kRec];
  float so[kTilePix * LPP / kWave][chunk_rows<LPP>()][KP + 4];  // padded like the record rows
  int flag;
};

// Whether batch entry l's ellipse can reach the wavefront's strip (entries past cnt: no).
template <class Sh>
__device__ __forceinline__ bool reaches(const Sh& S, int l, int cnt, float sx0, float sx1, float sy0, float sy1,
                                        float cut) {
  return l < cnt && S.mx[l] + S.hx[l] >= sx0 && S.mx[l] - S.hx[l] <= sx1 && S.my[l] + S.hy[l] >= sy0 &&
         S.my[l] - S.hy[l] <= sy1 && ellipse_meets(S.mx[l], S.my[l], S.qa[l], S.qb[l], S.qc[l], sx0, sx1, sy0, sy1, cut);
}

// Pass 1 of one tile: 256 lanes, one per pixel, four wavefronts of 16 x 4 strips, each walking
// the list on its own: lane l holds batch entry l in registers (the next batch is loaded
// while the current one is walked), the walk reads an entry's values with readlane, and a
// wavefront stops once all its pixels are done. Writes each pixel's final transmittance and
// last contributor (list position, -1 for none), claims a slot for every weighted Gaussian
// that contributes to a pixel (slot_of[g]: -1 until claimed; the claim takes it to -2 with a
// compare-and-swap, then to the slot from the counter), and per wavefront the list positions of its first contributor with a
// nonzero weight and of its last contributor (wave_range; INT_MAX / -1 when none): the back
// pass of a wavefront needs no entry outside that range, since only weighted contributors
// write records and only the contributors behind them feed their suffixes.
__global__ __launch_bounds__(kTilePix) void k_ig_front(
    const uint32_t* gids_, const uint32_t* ranges_, GroupCams gc, RasterConst rc, const float4* splat_,
    const float* __restrict__ conf, float* pix_t_, int32_t* pix_last_, int2* wave_range_, int32_t* slot_of_,
    int32_t* gid_of_, int32_t* n_slots_, int32_t* overflow_, int max_slots, int64_t* __restrict__ stats,
    const int32_t* tflag_, size_t vs) {
  const DevCam cam = gc.c[blockIdx.y];
  if ((int)blockIdx.x >= cam.tiles_x * cam.tiles_y) return;  // past this view's tiles
  const uint32_t* __restrict__ gids = vp(gids_, vs);
  const uint32_t* __restrict__ ranges = vp(ranges_, vs);
  const float4* __restrict__ splat = vp(splat_, vs);
  float* __restrict__ pix_t = vp(pix_t_, vs);
  int32_t* __restrict__ pix_last = vp(pix_last_, vs);
  int2* __restrict__ wave_range = vp(wave_range_, vs);
  int32_t* __restrict__ slot_of = vp(slot_of_, vs);
  int32_t* __restrict__ gid_of = vp(gid_of_, vs);
  int32_t* __restrict__ n_slots = vp(n_slots_, vs);
  int32_t* __restrict__ overflow = vp(overflow_, vs);
  const int32_t* __restrict__ tflag = vp(tflag_, vs);
  __shared__ int tile_last_sh;
  // with stats: the tile's list positions that contribute to some pixel (one bit per position,
  // the first kFBits of the list; beyond them each strip counts its own)
  constexpr int kFBits = 8192;
  __shared__ uint32_t fbits[kFBits / 32];
  const int ntiles = cam.tiles_x * cam.tiles_y;
  const int tile = blockIdx.x;
  if (tflag && tflag[tile] == 0) return;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int pix = threadIdx.x;
  const int px = tx * kTile + (pix & (kTile - 1));
  const int py = ty * kTile + (pix / kTile);
  const bool inside = px < cam.width && py < cam.height;
  const float fxp = (float)px + 0.5f, fyp = (float)py + 0.5f;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const uint32_t start = ranges[tile], end = ranges[ntiles + tile];
  const float sx0 = (float)(tx * kTile) + 0.5f, sx1 = sx0 + (float)(kTile - 1);
  const float sy0 = (float)(ty * kTile + wave * 4) + 0.5f, sy1 = sy0 + 3.f;
  if (stats) {
    for (int i = threadIdx.x; i < kFBits / 32; i += kTilePix) fbits[i] = 0u;
    __syncthreads();
  }
  uint32_t f_far = 0u;  // contributing positions beyond the bitmap (this strip)
  float T = 1.f;
  int last = -1, nc = 0;
  int wave_first = INT_MAX;
  bool done = !inside;
  // batch entry of this lane: gid and its walk record; the next two batches' are in flight
  // (a batch's walk is often short, and a record is a dependent gather behind its gid)
  uint32_t g1 = 0u, g2 = 0u;
  float4 a1 = make_float4(0.f, 0.f, 0.f, 0.f), b1 = make_float4(0.f, 0.f, 0.f, -1.f);
  float4 a2 = a1, b2 = b1;
  auto load = [&](uint32_t b, uint32_t& g, float4& ra, float4& rb) {
    if (b < end && lane < (int)(end - b)) {
      g = gids[b + lane];
      ra = splat[2 * (size_t)g];
      rb = splat[2 * (size_t)g + 1];
    }
  };
  load(start, g1, a1, b1);
  load(start + kWave, g2, a2, b2);
  for (uint32_t b0 = start; b0 < end; b0 += kWave) {
    if (__ballot(!done) == 0ull) break;
    const int cnt = (int)min((uint32_t)kWave, end - b0);
    const uint32_t eg = g1;
    const float emx = a1.x, emy = a1.y, eqa = a1.z, eqb = a1.w, eqc = b1.x, eop = b1.y;
    const float ehx = b1.z, ehy = b1.w;
    g1 = g2;
    a1 = a2;
    b1 = b2;
    load(b0 + 2 * kWave, g2, a2, b2);
    uint64_t live = __ballot(lane < cnt && emx + ehx >= sx0 && emx - ehx <= sx1 && emy + ehy >= sy0 &&
                             emy - ehy <= sy1 &&
                             ellipse_meets(emx, emy, eqa, eqb, eqc, sx0, sx1, sy0, sy1, rc.cutoff_q));
    uint64_t mine = 0ull;  // batch entries that contribute to this lane's pixel
    if (!done) {
      while (live) {
        const int j = __ffsll((unsigned long long)live) - 1;
        live &= live - 1;
        const float mxj = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, emx), j));
        const float myj = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, emy), j));
        const float qaj = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, eqa), j));
        const float qbj = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, eqb), j));
        const float qcj = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, eqc), j));
        const float opj = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, eop), j));
        const float dx = fxp - mxj, dy = fyp - myj;
        const float q = conic_q(qaj, qbj, qcj, dx, dy);
        if (q > rc.cutoff_q) continue;
        const float alpha = fminf(rc.alpha_max, gauss_alpha(opj, q));
        if (alpha < rc.alpha_min) continue;
        const float Tn = transmit(T, alpha);
        if (Tn < rc.t_min) { done = true; break; }
        T = Tn;
        last = (int)(b0 + j);
        ++nc;
        mine |= 1ull << j;
      }
    }
    // entries that contribute to some pixel of the wavefront: OR over the lanes' masks
    const uint64_t any = ((uint64_t)wave_or32((uint32_t)(mine >> 32)) << 32) | (uint64_t)wave_or32((uint32_t)mine);
    if (stats && any) {
      const uint32_t rel = b0 - start;  // a multiple of 64
      if (rel + kWave <= (uint32_t)kFBits) {
        if (lane == 0) {
          if ((uint32_t)any) atomicOr(&fbits[rel / 32], (uint32_t)any);
          if ((uint32_t)(any >> 32)) atomicOr(&fbits[rel / 32 + 1], (uint32_t)(any >> 32));
        }
      } else {
        f_far += (uint32_t)__popcll(any);
      }
    }
    bool weighted = false;
    if ((any >> lane) & 1ull) {
      weighted = conf[eg] > 0.f;
      // the first contribution of a weighted Gaussian claims its slot (past the capacity the
      // view overflows and the Gaussian stays unslotted)
      if (weighted && slot_of[eg] == -1 && atomicCAS(&slot_of[eg], -1, -2) == -1) {
        const int s = atomicAdd(n_slots, 1);
        if (s < max_slots) {
          gid_of[s] = (int32_t)eg;
          slot_of[eg] = s;
        } else {
          slot_of[eg] = -1;
          atomicOr(overflow, 1);
        }
      }
    }
    const uint64_t wm = __ballot(weighted);
    if (wave_first == INT_MAX && wm) wave_first = (int)b0 + __ffsll((unsigned long long)wm) - 1;
  }
  if (inside) {
    pix_t[(size_t)tile * kTilePix + pix] = T;
    pix_last[(size_t)tile * kTilePix + pix] = last;
  }
  int wave_last = last;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) wave_last = max(wave_last, __shfl_xor(wave_last, off));
  if (lane == 0) wave_range[(size_t)tile * (kTilePix / kWave) + wave] = make_int2(wave_first, wave_last);
  if (!stats) return;
  if (threadIdx.x == 0) tile_last_sh = -1;
  __syncthreads();
  if (last >= 0) atomicMax(&tile_last_sh, last);
  int tot = nc;
  for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
  if (lane == 0 && tot) atomicAdd((unsigned long long*)&stats[3], (unsigned long long)tot);
  // contributing (tile, Gaussian) pairs F
  uint32_t f = lane == 0 ? f_far : 0u;
  for (int i = threadIdx.x; i < kFBits / 32; i += kTilePix) f += (uint32_t)__popc(fbits[i]);
  for (int off = 32; off > 0; off >>= 1) f += __shfl_xor(f, off);
  if (lane == 0 && f) atomicAdd((unsigned long long*)&stats[9], (unsigned long long)f);
  __syncthreads();
  if (threadIdx.x == 0 && tile_last_sh >= 0)
    atomicAdd((unsigned long long*)&stats[4], (unsigned long long)(tile_last_sh - (int)start + 1));
}

// WPS: waves per SIMD the register allocation must allow (the launch bound): 3 with one lane
// per pixel, 1 with two or four (one 512- or 1024-lane workgroup per CU), or 4 for the
// two-lane variant that keeps two workgroups per CU at the cost of a few spilled registers.
template <int KP, int LPP, int WPS>
__global__ __launch_bounds__(kTilePix * LPP, WPS) void k_ig_back(
    int n, int k, const uint32_t* gids_, const uint32_t* ranges_, GroupCams gc, RasterConst rc, const float4* splat_,
    const float* depth_, const float* __restrict__ rgb, const float* __restrict__ prob, int obj_eq2, float* acc_,
    int astride, const int32_t* slot_of_, int64_t* __restrict__ stats, const int32_t* tflag_, const float* pix_t_,
    const int32_t* pix_last_, const int2* wave_range_, size_t vs) {
  const DevCam cam = gc.c[blockIdx.y];
  if ((int)blockIdx.x >= cam.tiles_x * cam.tiles_y) return;  // past this view's tiles
  const uint32_t* __restrict__ gids = vp(gids_, vs);
  const uint32_t* __restrict__ ranges = vp(ranges_, vs);
  const float4* __restrict__ splat = vp(splat_, vs);
  const float* __restrict__ depth = vp(depth_, vs);
  float* __restrict__ acc = vp(acc_, vs);
  const int32_t* __restrict__ slot_of = vp(slot_of_, vs);
  const int32_t* __restrict__ tflag = vp(tflag_, vs);
  const float* __restrict__ pix_t = vp(pix_t_, vs);
  const int32_t* __restrict__ pix_last = vp(pix_last_, vs);
  const int2* __restrict__ wave_range = vp(wave_range_, vs);
  extern __shared__ __align__(16) unsigned char smem_raw[];
  IgShared<KP, LPP>& S = *reinterpret_cast<IgShared<KP, LPP>*>(smem_raw);
  constexpr int kThreads = kTilePix * LPP;
  constexpr int kChunk = chunk_rows<LPP>();
  constexpr int KL = KP / LPP;           // object channels held per lane
  constexpr int kRowsW = kWave / LPP / kTile;  // pixel rows per wavefront
  // lanes of the wavefront that are the first of their pixel
  constexpr uint64_t kH0 = LPP == 1 ? ~0ull : (LPP == 2 ? 0x5555555555555555ull : 0x1111111111111111ull);
  const int ntiles = cam.tiles_x * cam.tiles_y;
  const int tile = blockIdx.x;
  // no weighted Gaussian reaches this tile: nothing of it enters a statistic
  if (tflag && tflag[tile] == 0) return;
  const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
  const int pix = threadIdx.x / LPP, h = threadIdx.x % LPP;  // pixel, and part of its channels
  const int px = tx * kTile + (pix & (kTile - 1));
  const int py = ty * kTile + (pix / kTile);
  const bool inside = px < cam.width && py < cam.height;
  const float fxp = (float)px + 0.5f, fyp = (float)py + 0.5f;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const uint32_t start = ranges[tile], end = ranges[ntiles + tile];
  // statistics owned by this lane in the reduction: scalar s = lane and 64 + lane (the
  // second one is dropped past the 94 scalars), Z_o channel zc of pixel group grp
  constexpr int kGroups = kWave / KP;
  const int zc = lane % KP, grp = lane / KP;
  const int sB = kWave + lane;
  const int ua = c_stats.d[lane].u, va = c_stats.d[lane].v;
  const int ub = sB < kStatScalar ? c_stats.d[sB].u : 0, vb = sB < kStatScalar ? c_stats.d[sB].v : 0;
  // pixel-centre bounds of this wavefront's 16 x kRowsW strip
  const float sx0 = (float)(tx * kTile) + 0.5f, sx1 = sx0 + (float)(kTile - 1);
  const float sy0 = (float)(ty * kTile + wave * kRowsW) + 0.5f, sy1 = sy0 + (float)(kRowsW - 1);

  // final transmittance and last contributor of this lane's pixel, and the list ranges of the
  // front pass's 16 x 4 strips: the tile's back pass runs from the last contributor of any of
  // its pixels to the first weighted contributor of any of them; a wavefront skips the entries
  // outside the range of the front strip that holds its rows (4 / LPP of them)
  float T = 1.f;
  int last = -1;
  if (inside) {
    T = pix_t[(size_t)tile * kTilePix + pix];
    last = pix_last[(size_t)tile * kTilePix + pix];
  }
  int tile_last = -1, first_w = INT_MAX, wave_first = INT_MAX, wave_last = -1;
  constexpr int kFrontWaves = kTilePix / kWave;  // 16 x 4 strips of the front pass
  for (int fw = 0; fw < kFrontWaves; ++fw) {
    const int2 r = wave_range[(size_t)tile * kFrontWaves + fw];
    tile_last = max(tile_last, r.y);
    first_w = min(first_w, r.x);
    if (fw == wave * kRowsW / 4) {
      wave_first = min(wave_first, r.x);
      wave_last = max(wave_last, r.y);
    }
  }
  if (tile_last < 0 || first_w > tile_last) return;
  if (stats && threadIdx.x == 0)
    atomicAdd((unsigned long long*)&stats[6], (unsigned long long)(tile_last - first_w + 1));

  // ---- pass 2: back to front ------------------------------------------------------------
  const float t_final = T;
  float Tc = T;
  float Sr = 0.f, Sg = 0.f, Sb = 0.f, Sd = 0.f;
  float So[KL];  // channels h * KL ... (h + 1) * KL - 1 of the object suffix
#pragma unroll
  for (int c = 0; c < KL; ++c) So[c] = 0.f;
  if (obj_eq2 && h == 0) So[0] = t_final;  // S~ = S_o + T_final e_0
  // counts for the statistics: contributing (pixel, entry) pairs of this pass and records
  uint32_t n_pass2 = 0u, n_rec = 0u;
  // with statistics: shader-clock cycles of this wavefront waiting at the batch barrier, staging
  // batches, walking them, and (part of the walk) reducing records
  const bool timed = stats != nullptr;
  uint64_t c_bar = 0u, c_load = 0u, c_walk = 0u, c_rec = 0u;
  constexpr int kBatch = batch_entries<LPP>();
  for (int hi = tile_last + 1; hi > first_w; hi -= kBatch) {
    const int lo = max(first_w, hi - kBatch);
    const int cnt = hi - lo;
    const uint64_t t_a = timed ? __builtin_amdgcn_s_memtime() : 0u;
    __syncthreads();
    const uint64_t t_b = timed ? __builtin_amdgcn_s_memtime() : 0u;
    if ((int)threadIdx.x < cnt) {
      const int j = threadIdx.x;
      const uint32_t g = gids[lo + j];
      const float4 a = splat[2 * (size_t)g], b = splat[2 * (size_t)g + 1];
      S.slot[j] = slot_of[g];
      S.mx[j] = a.x; S.my[j] = a.y; S.qa[j] = a.z; S.qb[j] = a.w;
      S.qc[j] = b.x; S.op[j] = b.y; S.hx[j] = b.z; S.hy[j] = b.w;
      S.z[j] = depth[g];
      S.r[j] = rgb[g]; S.g[j] = rgb[n + g]; S.b[j] = rgb[2 * n + g];
    }
    for (int idx = threadIdx.x; idx < cnt * KP; idx += kThreads) {
      const int j = idx / KP, c = idx % KP;
      S.p[j][c] = (c < k) ? prob[(size_t)gids[lo + j] * k + c] : 0.f;
    }
    __syncthreads();
    const uint64_t t_c = timed ? __builtin_amdgcn_s_memtime() : 0u;
    c_bar += t_b - t_a;
    c_load += t_c - t_b;
    uint64_t live =
        __ballot(lo + lane <= wave_last && lo + lane >= wave_first &&
                 reaches(S, lane, cnt, sx0, sx1, sy0, sy1, rc.cutoff_q));
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
        om = __builtin_amdgcn_rcpf(1.f - alpha);  // 1 ulp; 1 - alpha >= 0.01
        Tg = Tc * om;
        a = alpha * Tg;
      }
      const int slot = S.slot[j];
      const uint64_t cmask = __ballot(contrib);
      if (slot >= 0 && cmask) {
        const uint64_t t_r = timed ? __builtin_amdgcn_s_memtime() : 0u;
        // record of this lane's pixel (all zero when it does not contribute)
        float rv[kRec];
        {
          float y[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
          float wr = 0.f, wg = 0.f, wb = 0.f, wd = 0.f, nrgb = 0.f, no = 0.f;
          if (contrib) {
            if (raw < rc.alpha_max) {
              y[0] = alpha * (S.qa[j] * dx + S.qb[j] * dy);
              y[1] = alpha * (S.qb[j] * dx + S.qc[j] * dy);
              y[2] = -0.5f * alpha * dx * dx;
              y[3] = -alpha * dx * dy;
              y[4] = -0.5f * alpha * dy * dy;
              y[5] = alpha * (1.f - S.op[j]);
            }
            wr = S.r[j] * Tg - Sr * om;
            wg = S.g[j] * Tg - Sg * om;
            wb = S.b[j] * Tg - Sb * om;
            wd = S.z[j] * Tg - Sd * om;
            nrgb = wr * wr + wg * wg + wb * wb;
#pragma unroll
            for (int c = 0; c < KL; ++c) {
              const float w = S.p[j][h * KL + c] * Tg - So[c] * om;
              no += w * w;
            }
          }
#pragma unroll
          for (int off = 1; off < LPP; off <<= 1) no += __shfl_xor(no, off);
          const float ao = a * om, wd2 = wd * wd;
#pragma unroll
          for (int i = 0; i < 6; ++i) {
            rv[i] = y[i];
            rv[6 + i] = nrgb * y[i];
            rv[12 + i] = no * y[i];
            rv[18 + i] = wd2 * y[i];
            rv[kRecZ + i] = ao * y[i];
          }
          rv[kRecAW] = a * wr; rv[kRecAW + 1] = a * wg; rv[kRecAW + 2] = a * wb; rv[kRecAW + 3] = a * wd;
          rv[kRecAT] = a * Tg; rv[kRecA] = a;
        }
        // pixels (first lanes) that contribute; ranks of this lane's pixel among them and
        // among the others
        const uint64_t pmask = cmask & kH0;
        const int cnt = __popcll(pmask);
        n_rec += (uint32_t)cnt;
        const uint64_t below = (1ull << (lane - h)) - 1ull;
        const int rank = __popcll(pmask & below);
        const int nrank = __popcll(~pmask & kH0 & below);
        float (*rec)[kRec] = S.rec[wave];
        float (*sov)[KP + 4] = S.so[wave];
        float accA = 0.f, accB = 0.f, z[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        for (int c0 = 0; c0 < cnt; c0 += kChunk) {
          // rows [0, m) take the next contributing lanes; a short last chunk is padded to a
          // multiple of 4 rows with the (zero) records of non-contributing lanes
          const int m = min(kChunk, cnt - c0);
          const int R = (m + 3) & ~3;
          const int row = contrib ? rank - c0 : m + nrank;
          if (contrib ? (row >= 0 && row < m) : (row < R)) {
            if (h == 0) {
              float* dst = rec[row];
#pragma unroll
              for (int e = 0; e < kRec; e += 4) *reinterpret_cast<float4*>(dst + e) = make_float4(rv[e], rv[e + 1], rv[e + 2], rv[e + 3]);
            }
            float* srow = sov[row] + h * KL;
            if constexpr (KL % 4 == 0) {
#pragma unroll
              for (int c = 0; c < KL; c += 4)
                *reinterpret_cast<float4*>(srow + c) = make_float4(So[c], So[c + 1], So[c + 2], So[c + 3]);
            } else {
              // fewer than four channels per lane (k <= 4 with two lanes per pixel)
#pragma unroll
              for (int c = 0; c < KL; ++c) srow[c] = So[c];
            }
          }
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
          reduce_rows<KP>(R, rec, sov, ua, va, ub, vb, grp, zc, accA, accB, z);
          __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
          __builtin_amdgcn_wave_barrier();
          __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
#pragma unroll
        for (int off = KP; off < kWave; off <<= 1)
#pragma unroll
          for (int i = 0; i < 6; ++i) z[i] += __shfl_xor(z[i], off);
        float* dst = acc + (size_t)slot * astride;
        if (accA != 0.f) atomicAdd(dst + lane, accA);
        if (sB < kStatScalar && accB != 0.f) atomicAdd(dst + sB, accB);
        if (grp == 0 && zc < k) {
#pragma unroll
          for (int i = 0; i < 6; ++i)
            if (z[i] != 0.f) atomicAdd(dst + kStatScalar + i * k + zc, z[i]);
        }
        if (timed) c_rec += __builtin_amdgcn_s_memtime() - t_r;
      }
      if (contrib) {
        n_pass2 += h == 0 ? 1u : 0u;
        Sr += S.r[j] * a; Sg += S.g[j] * a; Sb += S.b[j] * a;
        Sd += S.z[j] * a;
#pragma unroll
        for (int c = 0; c < KL; ++c) So[c] += S.p[j][h * KL + c] * a;
        Tc = Tg;
      }
    }
    if (timed) c_walk += __builtin_amdgcn_s_memtime() - t_c;
  }
  if (stats) {
    uint32_t tot = n_pass2;
    for (int off = 32; off > 0; off >>= 1) tot += __shfl_xor(tot, off);
    if (lane == 0) {
      if (tot) atomicAdd((unsigned long long*)&stats[7], (unsigned long long)tot);
      if (n_rec) atomicAdd((unsigned long long*)&stats[8], (unsigned long long)n_rec);
      atomicAdd((unsigned long long*)&stats[10], (unsigned long long)c_bar);
      atomicAdd((unsigned long long*)&stats[11], (unsigned long long)c_load);
      atomicAdd((unsigned long long*)&stats[12], (unsigned long long)c_walk);
      atomicAdd((unsigned long long*)&stats[13], (unsigned long long)c_rec);
    }
  }
}

__global__ __launch_bounds__(256) void k_ig_clear(int32_t* n_slots_, int32_t* overflow_, int32_t* tflag_, GroupDims gd,
                                                  size_t vs) {
  int32_t* n_slots = vp(n_slots_, vs);
  int32_t* overflow = vp(overflow_, vs);
  int32_t* tflag = vp(tflag_, vs);
  const int ntiles = gd.tx[blockIdx.y] * gd.ty[blockIdx.y];
  if (threadIdx.x == 0) {
    *n_slots = 0;
    *overflow = 0;
  }
  if (tflag)
    for (int i = threadIdx.x; i < ntiles; i += blockDim.x) tflag[i] = 0;
}

// With a target object: flags the tiles that the rect of a weighted Gaussian (nonzero
// confidence, reaching a tile) covers, so that both passes and the filtered binning can leave
// the other tiles at once. A wavefront marks the rects of its weighted Gaussians together,
// one Gaussian at a time; the cost is the rect areas of the weighted Gaussians, small when only
// one object carries weight.
__global__ __launch_bounds__(256) void k_ig_mark(int n, const float* __restrict__ conf, const uint32_t* count_,
                                                 const int16_t* rect_, int32_t* tflag_, GroupDims gd, size_t vs) {
  const uint32_t* __restrict__ count = vp(count_, vs);
  const int16_t* __restrict__ rect = vp(rect_, vs);
  int32_t* __restrict__ tflag = vp(tflag_, vs);
  const int tiles_x = gd.tx[blockIdx.y], tiles_y = gd.ty[blockIdx.y];
  const int lane = threadIdx.x % kWave;
  const int g = blockIdx.x * 256 + threadIdx.x;
  const bool weighted = g < n && count[g] > 0u && conf[g] > 0.f;
  // each lane's rect is loaded up front (the loop below only stores: no load waits behind them)
  int2 rr = make_int2(0, -1);
  if (weighted) rr = reinterpret_cast<const int2*>(rect)[g];
  uint64_t m = __ballot(weighted);
  while (m) {
    const int j = __ffsll((unsigned long long)m) - 1;
    m &= m - 1;
    const int r01 = __builtin_amdgcn_readlane(rr.x, j), r23 = __builtin_amdgcn_readlane(rr.y, j);
    const int x0 = max((int)(int16_t)(r01 & 0xFFFF), 0), y0 = max(r01 >> 16, 0);
    const int x1 = min((int)(int16_t)(r23 & 0xFFFF), tiles_x - 1), y1 = min(r23 >> 16, tiles_y - 1);
    if (x1 < x0 || y1 < y0) continue;
    const int w = x1 - x0 + 1, area = w * (y1 - y0 + 1);
    for (int t = lane; t < area; t += kWave) tflag[(y0 + t / w) * tiles_x + x0 + t % w] = 1;
  }
}

// Zero the statistic rows of the assigned slots.
__global__ __launch_bounds__(256) void k_ig_zero(float4* acc_, const int32_t* n_slots_, int max_slots, int astride,
                                                 size_t vs) {
  float4* __restrict__ acc = vp(acc_, vs);
  const int32_t* __restrict__ n_slots = vp(n_slots_, vs);
  const size_t total = (size_t)min(*n_slots, max_slots) * (size_t)(astride / 4);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x)
    acc[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

template <int KP, int LPP, int WPS = (3 / LPP > 0 ? 3 / LPP : 1)>
hipError_t launch_ig_k(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l, const Group& G,
                       const RasterConst& rc, const ngs_ig_params& ig, const IgWs& w, const int32_t* tflag, int64_t* stats,
                       hipStream_t st) {
  const int ntiles = G.max_ntiles;
  const size_t shm = sizeof(IgShared<KP, LPP>);
  static_assert(sizeof(IgShared<KP, LPP>) <= 65536, "IG kernel LDS");
  ProfScope ps(kProfIgTiles, st);
  hipLaunchKernelGGL((k_ig_back<KP, LPP, WPS>), dim3(ntiles, G.g), dim3(kTilePix * LPP), shm, st, s.n, s.k, l.gids,
                     l.ranges, G.cams, rc, reinterpret_cast<const float4*>(p.splat), p.depth, s.rgb, s.prob, ig.obj_eq2,
                     w.acc, w.astride, w.slot_of, stats, tflag, w.pix_t, w.pix_last, w.wave_range, G.vs);
  return hipGetLastError();
}

}  // namespace

int ig_stat_stride(int64_t k) { return (stat_len((int)k) + 15) / 16 * 16; }

size_t ig_ws_fixed_bytes(int64_t n) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  return al(nn * 4) + al(8) + al((size_t)NGS_MAX_TILES * 4) + 2 * al((size_t)NGS_MAX_TILES * kTilePix * 4) +
         al((size_t)NGS_MAX_TILES * (kTilePix / kWave) * 8);
}

size_t ig_ws_bytes(int64_t n, int64_t k, int64_t max_slots) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  return al((size_t)ig_stat_stride(k) * (size_t)max_slots * 4) + al((size_t)max_slots * 4) + ig_ws_fixed_bytes(n) +
         al((size_t)max_slots * 7 * kNGeo * 8);
}

IgWs ig_ws_carve(void* ws, int64_t n, int64_t k, int64_t max_slots) {
  auto al = [](size_t x) { return (x + 255) / 256 * 256; };
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  char* p = static_cast<char*>(ws);
  IgWs w;
  w.astride = ig_stat_stride(k);
  w.acc = (float*)p; p += al((size_t)w.astride * (size_t)max_slots * 4);
  w.slot_of = (int32_t*)p; p += al(nn * 4);
  w.gid_of = (int32_t*)p; p += al((size_t)max_slots * 4);
  w.n_slots = (int32_t*)p; p += al(8);
  w.overflow = w.n_slots + 1;
  w.tflag = (int32_t*)p; p += al((size_t)NGS_MAX_TILES * 4);
  w.pix_t = (float*)p; p += al((size_t)NGS_MAX_TILES * kTilePix * 4);
  w.pix_last = (int32_t*)p; p += al((size_t)NGS_MAX_TILES * kTilePix * 4);
  w.wave_range = (int2*)p; p += al((size_t)NGS_MAX_TILES * (kTilePix / kWave) * 8);
  w.pmat = (double*)p;
  w.max_slots = max_slots;
  return w;
}

const int32_t* ig_tile_flags(const ngs_ig_params& ig, const IgWs& w) {
  // Tile flags only pay when few Gaussians carry weight (one target object, Eq. 12); with
  // whole-scene confidence nearly every tile holds a weighted Gaussian.
  return ig.target_id >= 0 ? w.tflag : nullptr;
}

hipError_t launch_ig_clear(const ngs_ig_params& ig, const IgWs& w, const Group& G, hipStream_t st) {
  int32_t* tflag = const_cast<int32_t*>(ig_tile_flags(ig, w));
  ProfScope ps(kProfFill, st);
  hipLaunchKernelGGL(k_ig_clear, dim3(1, G.g), dim3(256), 0, st, w.n_slots, w.overflow, tflag, G.dims, G.vs);
  return hipGetLastError();
}

hipError_t launch_ig_assign(const ngs_scene& s, const ngs_projected& p, const Group& G, const ngs_ig_params& ig,
                            const IgWs& w, hipStream_t st) {
  int32_t* tflag = const_cast<int32_t*>(ig_tile_flags(ig, w));
  hipError_t e = launch_ig_clear(ig, w, G, st);
  if (e != hipSuccess) return e;
  if (tflag && s.n > 0) {
    ProfScope ps(kProfIgAssign, st);
    hipLaunchKernelGGL(k_ig_mark, dim3((s.n + 255) / 256, G.g), dim3(256), 0, st, s.n, s.conf, p.count, p.rect, tflag,
                       G.dims, G.vs);
  }
  return hipGetLastError();
}

hipError_t launch_ig_reset_slots(const IgWs& w, int64_t n, hipStream_t st) {
  return launch_fill_u32(reinterpret_cast<uint32_t*>(w.slot_of), 0xFFFFFFFFu, (size_t)std::max<int64_t>(n, 1), st, 1,
                         0);
}

hipError_t launch_ig_walk(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l, const Group& G,
                          const RasterConst& rc, const ngs_ig_params& ig, const IgWs& w, int64_t* stats, int lpp,
                          hipStream_t st, int waves) {
  const int32_t* tflag = ig_tile_flags(ig, w);
  {
    ProfScope ps(kProfIgFront, st);
    hipLaunchKernelGGL(k_ig_front, dim3(G.max_ntiles, G.g), dim3(kTilePix), 0, st, l.gids, l.ranges, G.cams, rc,
                       reinterpret_cast<const float4*>(p.splat), s.conf, w.pix_t, w.pix_last, w.wave_range, w.slot_of,
                       w.gid_of, w.n_slots, w.overflow, (int)w.max_slots, stats, tflag, G.vs);
  }
  {
    ProfScope ps(kProfIgAssign, st);
    hipLaunchKernelGGL(k_ig_zero, dim3(std::max(64, 1024 / G.g), G.g), dim3(256), 0, st,
                       reinterpret_cast<float4*>(w.acc), w.n_slots, (int)w.max_slots, w.astride, G.vs);
  }
  // lanes per pixel (ig_lpp_valid): 0 picks the default of each object-vector width
  if (s.k <= 4) return lpp == 2 ? launch_ig_k<4, 2>(s, p, l, G, rc, ig, w, tflag, stats, st)
                                : launch_ig_k<4, 1>(s, p, l, G, rc, ig, w, tflag, stats, st);
  if (s.k <= 8) return lpp == 2 ? launch_ig_k<8, 2>(s, p, l, G, rc, ig, w, tflag, stats, st)
                                : launch_ig_k<8, 1>(s, p, l, G, rc, ig, w, tflag, stats, st);
  if (s.k <= 16) return lpp == 1 ? launch_ig_k<16, 1>(s, p, l, G, rc, ig, w, tflag, stats, st)
                        : lpp == 4 ? launch_ig_k<16, 4>(s, p, l, G, rc, ig, w, tflag, stats, st)
                                   : launch_ig_k<16, 2>(s, p, l, G, rc, ig, w, tflag, stats, st);
  if (s.k <= 32) return lpp == 1 ? launch_ig_k<32, 1>(s, p, l, G, rc, ig, w, tflag, stats, st)
                        : lpp == 4 ? launch_ig_k<32, 4>(s, p, l, G, rc, ig, w, tflag, stats, st)
                        : waves == 4 ? launch_ig_k<32, 2, 4>(s, p, l, G, rc, ig, w, tflag, stats, st)
                                     : launch_ig_k<32, 2>(s, p, l, G, rc, ig, w, tflag, stats, st);
  return lpp == 1 ? launch_ig_k<64, 1>(s, p, l, G, rc, ig, w, tflag, stats, st)
         : waves == 4 ? launch_ig_k<64, 2, 4>(s, p, l, G, rc, ig, w, tflag, stats, st)
                      : launch_ig_k<64, 2>(s, p, l, G, rc, ig, w, tflag, stats, st);
}

hipError_t launch_ig_tiles(const ngs_scene& s, const ngs_projected& p, const ngs_tile_lists& l, const Group& G,
                           const RasterConst& rc, const ngs_ig_params& ig, const IgWs& w, int64_t* stats, int lpp,
                           hipStream_t st, int waves) {
  hipError_t e = launch_ig_assign(s, p, G, ig, w, st);
  if (e != hipSuccess) return e;
  return launch_ig_walk(s, p, l, G, rc, ig, w, stats, lpp, st, waves);
}

bool ig_lpp_valid(int64_t k, int lpp) {
  if (lpp == 0) return true;
  if (k <= 8) return lpp == 1 || lpp == 2;
  if (k <= 32) return lpp == 1 || lpp == 2 || lpp == 4;
  return lpp == 1 || lpp == 2;
}

bool ig_waves_valid(int64_t k, int lpp, int waves) {
  if (waves == 0) return true;
  const int l = lpp == 0 ? (k <= 8 ? 1 : 2) : lpp;
  return waves == 4 && l == 2 && k > 16;
}

}  // namespace ngs
