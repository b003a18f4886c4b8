// bin.hip -- tile binning: (tile, depth, gid)-sorted lists of every (tile, Gaussian) pair.
//
// The sort is an LSD radix sort on the composite key (tile, float32 depth bits, gid) run in
// two stages, because all pairs of one Gaussian share its depth bits:
//   1. depth digits: the n Gaussians are sorted by their 32-bit depth key (4 passes over n
//      entries instead of over the M >> n pairs); gid order breaks ties (stable LSD);
//   2. the tile digit in two stable counting levels fused with the pairs' generation:
//      level 1 places one entry per (row of tiles, Gaussian) - gid and the Gaussian's tile
//      span x0, w - into per-row segments in depth order (single-wavefront blocks of 512
//      consecutive depth ranks; count, scan over blocks, scatter); level 2 splits every
//      row's segment into chunks and places each entry's pairs into the row's tiles (count
//      per (tile, chunk), scan over the row's chunks, scatter). A scatter takes 64 entries
//      at a time, one per lane in depth order, and for each row (tile) they cover ranks the
//      covering lanes with a ballot, so every level is stable and each write is a run.
// The result equals a sort of (tile << 32 | depth bits) with ties broken by gid; the
// per-tile ranges fall out of the scan. A single level over all tiles (a block writing ~10
// pairs into each of ~1,200 tiles) left thousands of half-written lines per block in the
// L2 and wrote ~8x the pairs' bytes to HBM; level 2's blocks touch only one row's tiles.
#include "common.hpp"

namespace ngs {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;  // counts summed per block

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// The view's pair count M = sum of the per-Gaussian tile counts, in two launches with no
// atomics: block partials, then one block per view adds them up in order.
__global__ __launch_bounds__(kScanThreads) void k_count_partials(const uint32_t* count_, int n, uint64_t* bsum_,
                                                                 size_t vs) {
  const uint32_t* __restrict__ count = vp(count_, vs);
  uint64_t* __restrict__ bsum = vp(bsum_, vs);
  __shared__ uint64_t sm[kScanThreads / kWave];
  const int t = threadIdx.x;
  uint64_t v = 0ull;
  for (int j = 0; j < kScanItems; ++j) {
    const int i = blockIdx.x * kScanTile + j * kScanThreads + t;
    if (i < n) v += count[i];
  }
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (t % kWave == 0) sm[t / kWave] = v;
  __syncthreads();
  if (t == 0) {
    uint64_t s = 0ull;
    for (int w = 0; w < kScanThreads / kWave; ++w) s += sm[w];
    bsum[blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(kScanThreads) void k_count_total(const uint64_t* bsum_, int nb, uint64_t* total_,
                                                              size_t vs) {
  const uint64_t* __restrict__ bsum = vp(bsum_, vs);
  uint64_t* __restrict__ total = vp(total_, vs);
  __shared__ uint64_t sm[kScanThreads / kWave];
  const int t = threadIdx.x;
  uint64_t v = 0ull;
  for (int i = t; i < nb; i += kScanThreads) v += bsum[i];
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (t % kWave == 0) sm[t / kWave] = v;
  __syncthreads();
  if (t == 0) {
    uint64_t s = 0ull;
    for (int w = 0; w < kScanThreads / kWave; ++w) s += sm[w];
    *total = s;
  }
}

constexpr int kPartRanks = 512;  // depth ranks per level-1 partition block (one wavefront)
constexpr int kChunk2 = 512;     // least row entries per level-2 chunk (default; tunable)
constexpr int kHist2 = 1 << 22;  // level-2 count table entries (tiles_x * chunks)
constexpr int kGrid2 = 8192;     // persistent level-2 wavefronts
constexpr int kWaves2 = 4;       // independent wavefronts per level-2 workgroup

// One Gaussian's rect as seen by the whole wavefront: lane q's values broadcast.
struct RectU {
  uint32_t gid;
  int x0, y0, w, area;
  float inv_w;
};

// A lane's Gaussian of rank r: gid, tile origin packed as x0 | y0 << 16, width, area and
// 1 / width (area 0 past n or for a culled Gaussian).
struct RectL {
  uint32_t gid, org;
  int w, area;
  float inv_w;
};

// What a lane loads for depth rank r (past n: an empty rect), and the rect it describes.
struct RectRaw {
  uint32_t gid;
  short4 b;
};
__device__ __forceinline__ RectRaw part_lane_raw(int n, int r, const uint32_t* __restrict__ order,
                                                 const int16_t* __restrict__ rect_sorted) {
  RectRaw q{0u, make_short4(0, 0, -1, -1)};
  if (r < n) {
    q.gid = order[r];
    q.b = reinterpret_cast<const short4*>(rect_sorted)[r];
  }
  return q;
}
__device__ __forceinline__ RectL part_lane_rect(const RectRaw& q) {
  RectL l;
  l.gid = q.gid;
  l.org = (uint32_t)(uint16_t)q.b.x | ((uint32_t)(uint16_t)q.b.y << 16);
  l.w = q.b.z - q.b.x + 1;
  l.area = q.b.z >= q.b.x ? l.w * (q.b.w - q.b.y + 1) : 0;
  l.w = l.area > 0 ? l.w : 1;
  l.inv_w = 1.f / (float)l.w;
  return l;
}

__device__ __forceinline__ RectU part_bcast(const RectL& l, int q) {
  RectU u;
  u.gid = (uint32_t)__builtin_amdgcn_readlane((int)l.gid, q);
  const uint32_t org = (uint32_t)__builtin_amdgcn_readlane((int)l.org, q);
  u.x0 = (int)(org & 0xFFFFu);
  u.y0 = (int)(org >> 16);
  u.w = __builtin_amdgcn_readlane(l.w, q);
  u.area = __builtin_amdgcn_readlane(l.area, q);
  u.inv_w = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, l.inv_w), q));
  return u;
}

// Rank chunk of partition block b. Workgroups are dealt to the 8 XCDs round robin, so
// block b runs on XCD b % 8; giving each XCD a contiguous range of chunks keeps adjacent
// pieces of every tile's output segment (and of the count table) in one L2.
__device__ __forceinline__ int part_chunk(int b, int nblk) {
  constexpr int kXcd = 8;
  const int x = b % kXcd, q = nblk / kXcd, r = nblk % kXcd;
  return x * q + min(x, r) + b / kXcd;
}

// Tile of entry j (row-major) of the rect. (j + 0.5) / w lies at least 0.5 / w from an
// integer; with j < 4096 the FP32 product errs by less than 4096 * 2^-23 / w, far inside
// that margin, so the truncation gives the exact row.
__device__ __forceinline__ int part_tile(const RectU& u, int j, int tiles_x) {
  const int row = (int)(((float)j + 0.5f) * u.inv_w);
  return (u.y0 + row) * tiles_x + u.x0 + (j - row * u.w);
}

// Per row of a (row, block) count table: exclusive scan across blocks (in place); totals.
__global__ __launch_bounds__(256) void k_part_scan_rows(uint32_t* hist_, int nblk, uint32_t* tot_, GroupDims gd,
                                                        size_t vs) {
  if ((int)blockIdx.x >= gd.ty[blockIdx.y]) return;  // past this view's rows
  uint32_t* __restrict__ hist = vp(hist_, vs);
  uint32_t* __restrict__ tot = vp(tot_, vs);
  __shared__ uint32_t sm[256];
  uint32_t* row = hist + (size_t)blockIdx.x * nblk;
  uint32_t carry = 0;
  for (int b0 = 0; b0 < nblk; b0 += 256) {
    const int i = b0 + threadIdx.x;
    const uint32_t v = (i < nblk) ? row[i] : 0u;
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const uint32_t add = (threadIdx.x >= (unsigned)off) ? sm[threadIdx.x - off] : 0u;
      __syncthreads();
      sm[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nblk) row[i] = carry + sm[threadIdx.x] - v;
    carry += sm[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = carry;
}

// Tile starts (exclusive scan of the per-tile totals) -> ranges; an empty tile gets
// start = end = the number of pairs in lower tiles. If the pairs (m_total, the sum of the
// tile counts) exceed the list capacity, every range is left empty and *overflow is raised (the
// scatters then write nothing).
__global__ __launch_bounds__(256) void k_part_ranges(const uint32_t* tot_, GroupDims gd, uint32_t* ranges_,
                                                     int64_t capacity, int32_t* __restrict__ overflow,
                                                     int64_t* __restrict__ stats, const uint64_t* m_total_,
                                                     const int32_t* keep_, size_t vs) {
  const uint32_t* __restrict__ tot = vp(tot_, vs);
  uint32_t* __restrict__ ranges = vp(ranges_, vs);
  const uint64_t* __restrict__ m_total = vp(m_total_, vs);
  const int32_t* __restrict__ keep = vp(keep_, vs);
  const int ntiles = gd.tx[blockIdx.y] * gd.ty[blockIdx.y];
  __shared__ uint32_t sm[256];
  constexpr int kPer = NGS_MAX_TILES / 256;
  const int t0 = threadIdx.x * kPer;
  uint32_t v[kPer];
  uint32_t run = 0;
  for (int j = 0; j < kPer; ++j) {
    v[j] = run;
    run += (t0 + j < ntiles) ? tot[t0 + j] : 0u;
  }
  sm[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t add = (threadIdx.x >= (unsigned)off) ? sm[threadIdx.x - off] : 0u;
    __syncthreads();
    sm[threadIdx.x] += add;
    __syncthreads();
  }
  const uint64_t total = *m_total;
  const bool over = (int64_t)total > capacity;
  const uint32_t excl = sm[threadIdx.x] - run;
  for (int j = 0; j < kPer; ++j)
    if (t0 + j < ntiles) {
      ranges[t0 + j] = over ? 0u : excl + v[j];
      ranges[ntiles + t0 + j] = over ? 0u : excl + v[j] + (keep && keep[t0 + j] == 0 ? 0u : tot[t0 + j]);
    }
  if (threadIdx.x == 0) {
    if (over && overflow) atomicOr(overflow, 1);
    if (stats) atomicAdd((unsigned long long*)&stats[1], (unsigned long long)total);
  }
}

// Bins [64 i2, 64 i2 + 64) covered by the span [b0, b0 + len), as bits.
__device__ __forceinline__ uint64_t span_bits(int b0, int len, int i2) {
  const int a = max(b0 - i2 * kWave, 0), b = min(b0 + len - i2 * kWave, kWave);
  if (len <= 0 || a >= b) return 0ull;
  return (b - a == kWave ? ~0ull : ((1ull << (b - a)) - 1ull)) << a;
}

// ---- wanted entries --------------------------------------------------------------------------
// With keep flags (tiles_x <= 128), a row entry whose span reaches no wanted tile of its row is
// not binned at all: both row passes apply the same test, so the wanted tiles' lists are those of
// the full binning. Row y's wanted tiles: bit x % 64 of rkm[2 y + x / 64].
__global__ __launch_bounds__(256) void k_keep_rows(const int32_t* keep_, GroupDims gd, unsigned long long* rkm_,
                                                   size_t vs) {
  const int32_t* __restrict__ keep = vp(keep_, vs);
  unsigned long long* __restrict__ rkm = vp(rkm_, vs);
  const int rows = gd.ty[blockIdx.y], tiles_x = gd.tx[blockIdx.y];
  for (int y = threadIdx.x; y < rows; y += blockDim.x) {
    unsigned long long m0 = 0ull, m1 = 0ull;
    for (int x = 0; x < tiles_x; ++x)
      if (keep[y * tiles_x + x] != 0) {
        if (x < 64) m0 |= 1ull << x;
        else m1 |= 1ull << (x - 64);
      }
    rkm[2 * y] = m0;
    rkm[2 * y + 1] = m1;
  }
}

// Row masks of the view in LDS (rows <= 128), and whether row r of a span whose tiles are
// (m0, m1) (span_bits of its x range) holds a wanted tile.
__device__ __forceinline__ void load_row_masks(unsigned long long* rk_sh, const unsigned long long* rkm, int rows) {
  for (int i = threadIdx.x; i < 2 * rows; i += blockDim.x) rk_sh[i] = rkm[i];
  __syncthreads();
}
__device__ __forceinline__ bool row_wanted(const unsigned long long* rk_sh, int r, uint64_t m0, uint64_t m1) {
  return ((m0 & rk_sh[2 * r]) | (m1 & rk_sh[2 * r + 1])) != 0ull;
}

// ---- level 1: rows ------------------------------------------------------------------------
// Pass 1a: row entries per (row, block), row-major: rhist[r * nblk + block]. Counting needs
// no order, so each lane adds its own Gaussian's rows.
__global__ __launch_bounds__(kWave) void k_row_hist(int n, const uint32_t* order_, const int16_t* rect_,
                                                    GroupDims gd, uint32_t* rhist_, int nblk,
                                                    const unsigned long long* rkm_, size_t vs) {
  const uint32_t* __restrict__ order = vp(order_, vs);
  const int16_t* __restrict__ rect = vp(rect_, vs);
  uint32_t* __restrict__ rhist = vp(rhist_, vs);
  const unsigned long long* __restrict__ rkm = vp(rkm_, vs);
  const int rows = gd.ty[blockIdx.y];
  extern __shared__ uint32_t cnt[];  // [rows]
  __shared__ unsigned long long rk_sh[2 * 2 * kWave];
  const int lane = threadIdx.x;
  const int chunk = part_chunk(blockIdx.x, nblk);
  for (int t = lane; t < rows; t += kWave) cnt[t] = 0u;
  if (rkm) load_row_masks(rk_sh, rkm, rows);
  __syncthreads();
  const int r0 = chunk * kPartRanks;
  // all of the block's entries are loaded before the first is used (one wait for them all;
  // in the scatter a wait for loads issued after stores would also wait for the stores)
  constexpr int kSub = kPartRanks / kWave;
  RectRaw raw[kSub];
#pragma unroll
  for (int q = 0; q < kSub; ++q) raw[q] = part_lane_raw(n, r0 + q * kWave + lane, order, rect);
  // one sub-batch at a time from raw[0], the rest moving down (static register indices)
#pragma unroll 1
  for (int q = 0; q < kSub; ++q) {
    if (r0 + q * kWave >= n) break;
    const RectL l = part_lane_rect(raw[0]);
#pragma unroll
    for (int t = 0; t + 1 < kSub; ++t) raw[t] = raw[t + 1];
    const int y0 = (int)(l.org >> 16), h = l.area / l.w, x0 = (int)(l.org & 0xFFFFu);
    if (rkm) {
      const uint64_t m0 = span_bits(x0, l.w, 0), m1 = span_bits(x0, l.w, 1);
      for (int j = 0; j < h; ++j)
        if (row_wanted(rk_sh, y0 + j, m0, m1)) atomicAdd(&cnt[y0 + j], 1u);
    } else {
      for (int j = 0; j < h; ++j) atomicAdd(&cnt[y0 + j], 1u);
    }
  }
  __syncthreads();
  for (int t = lane; t < rows; t += kWave) rhist[(size_t)t * nblk + chunk] = cnt[t];
}

// Pass 1b (one block): row starts, the level-2 chunking and the overflow decision.
// meta: [0] M (all pairs), [1] entries per level-2 chunk K2, [2] chunks NC, [3] over.
// K2 keeps the level-2 count table within kHist2 entries: tiles_x * NC <= kHist2.
__global__ __launch_bounds__(256) void k_row_starts(const uint32_t* rtot_, GroupDims gd, const uint64_t* m_total_,
                                                    int64_t capacity, uint32_t* rstart_, uint32_t* nch_, uint32_t* cp_,
                                                    uint32_t* meta_, int64_t* n_pairs_, uint32_t chunk_min, size_t vs) {
  const uint32_t* __restrict__ rtot = vp(rtot_, vs);
  const uint64_t* __restrict__ m_total = vp(m_total_, vs);
  uint32_t* __restrict__ rstart = vp(rstart_, vs);
  uint32_t* __restrict__ nch = vp(nch_, vs);
  uint32_t* __restrict__ cp = vp(cp_, vs);
  uint32_t* __restrict__ meta = vp(meta_, vs);
  int64_t* __restrict__ n_pairs = vp(n_pairs_, vs);
  const int rows = gd.ty[blockIdx.y], tiles_x = gd.tx[blockIdx.y];
  __shared__ uint32_t sm[256];
  __shared__ uint32_t k2_sh;
  constexpr int kPer = NGS_MAX_TILES / 256;
  const int t0 = threadIdx.x * kPer;
  const uint64_t M = *m_total;
  const bool over = (int64_t)M > capacity;
  // row starts
  uint32_t v[kPer];
  uint32_t run = 0;
  for (int j = 0; j < kPer; ++j) {
    v[j] = run;
    run += (t0 + j < rows && !over) ? rtot[t0 + j] : 0u;
  }
  sm[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t add = (threadIdx.x >= (unsigned)off) ? sm[threadIdx.x - off] : 0u;
    __syncthreads();
    sm[threadIdx.x] += add;
    __syncthreads();
  }
  const uint32_t m1 = sm[255];
  const uint32_t excl = sm[threadIdx.x] - run;
  for (int j = 0; j < kPer; ++j)
    if (t0 + j < rows) rstart[t0 + j] = excl + v[j];
  if (threadIdx.x == 0) {
    const uint64_t room = (uint64_t)kHist2 / (uint64_t)tiles_x - (uint64_t)rows;  // >= 1, see kHist2
    const uint64_t k2 = ((uint64_t)m1 + room - 1) / room;
    k2_sh = (uint32_t)(k2 > (uint64_t)chunk_min ? k2 : (uint64_t)chunk_min);
  }
  __syncthreads();
  const uint32_t K2 = k2_sh;
  __syncthreads();
  // chunks per row and their exclusive scan
  run = 0;
  for (int j = 0; j < kPer; ++j) {
    v[j] = run;
    run += (t0 + j < rows && !over) ? (rtot[t0 + j] + K2 - 1) / K2 : 0u;
  }
  sm[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t add = (threadIdx.x >= (unsigned)off) ? sm[threadIdx.x - off] : 0u;
    __syncthreads();
    sm[threadIdx.x] += add;
    __syncthreads();
  }
  const uint32_t excl2 = sm[threadIdx.x] - run;
  for (int j = 0; j < kPer; ++j)
    if (t0 + j < rows) {
      cp[t0 + j] = excl2 + v[j];
      nch[t0 + j] = (!over) ? (rtot[t0 + j] + K2 - 1) / K2 : 0u;
    }
  if (threadIdx.x == 0) {
    *n_pairs = (int64_t)M;
    cp[rows] = sm[255];
    meta[0] = (uint32_t)min(M, (uint64_t)0xFFFFFFFFu);
    meta[1] = K2;
    meta[2] = sm[255];
    meta[3] = over ? 1u : 0u;
  }
}

// Wave-wide min and max.
__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) v = min(v, __shfl_xor(v, off));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) v = max(v, __shfl_xor(v, off));
  return v;
}

// Places the current 64 entries (lane order = depth order) of one segment family: for every
// bin c in [lo, hi], the lanes that cover c (covers(c): c in the lane's span, and wanted) take consecutive positions
// cnt[c] + (covering lanes below them), and cnt[c] advances by their number. No atomics:
// ballots give the ranks, and each bin's writes are one coalesced run.
// Bins for which keep(c) is false are passed over: nothing is written for them and their
// counters stay as they were.
template <class Emit, class Keep, class Covers>
__device__ __forceinline__ void place_batch(uint32_t* cnt, int lo, int hi, int lane, Emit emit, Keep keep,
                                            Covers covers) {
  const uint64_t below = (1ull << lane) - 1ull;
  for (int c = lo; c <= hi; ++c) {
    if (!keep(c)) continue;
    const bool cover = covers(c);
    const uint64_t m = __ballot(cover);
    if (!m) continue;
    const uint32_t base = cnt[c];
    if (cover) emit(c, base + (uint32_t)__popcll(m & below));
    if (lane == 0) cnt[c] = base + (uint32_t)__popcll(m);
  }
}

// place_batch with the counters in registers (lane l holds bin 64 i2 + l in cr[i2], read with
// readlane at the uniform bin), over the bins that some lane covers: u[i2] holds this lane's
// bins of word i2 (bit c % 64 of word c / 64). The union of the 64 lanes' bins (OR over the wavefront) is
// walked bit by bit, so only bins that receive entries are visited (the bins of 64 depth-ordered
// entries leave gaps, and unwanted bins are masked out of u by the caller).
template <int NR, class Emit>
__device__ __forceinline__ void place_batch_masked(uint32_t (&cr)[NR], const uint64_t (&u)[NR], Emit emit) {
#pragma unroll
  for (int i2 = 0; i2 < NR; ++i2) {
    uint64_t todo = ((uint64_t)wave_or32((uint32_t)(u[i2] >> 32)) << 32) | (uint64_t)wave_or32((uint32_t)u[i2]);
    while (todo) {
      const int bit = __builtin_ctzll(todo);
      todo &= todo - 1ull;
      const bool cover = (u[i2] >> bit) & 1ull;
      const uint64_t m = __ballot(cover);
      const uint32_t base = (uint32_t)__builtin_amdgcn_readlane((int)cr[i2], bit);
      // base + the covering lanes below this one
      if (cover) emit(i2 * kWave + bit, __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, base)));
      if ((int)__lane_id() == bit) cr[i2] = base + (uint32_t)__popcll(m);
    }
  }
}

// Pass 1c: every Gaussian's row entries {gid, x0 | w << 16} to their row segments, in depth
// order within a row. NR > 0: counters in registers (rows <= 64 NR), else in LDS.
template <int NR>
__global__ __launch_bounds__(kWave) void k_row_scatter(int n, const uint32_t* order_, const int16_t* rect_,
                                                       GroupDims gd, const uint32_t* rhist_, int nblk,
                                                       const uint32_t* rstart_, const uint32_t* meta_, uint2* rl_,
                                                       const unsigned long long* rkm_, size_t vs) {
  const uint32_t* __restrict__ order = vp(order_, vs);
  const int16_t* __restrict__ rect = vp(rect_, vs);
  const uint32_t* __restrict__ rhist = vp(rhist_, vs);
  const uint32_t* __restrict__ rstart = vp(rstart_, vs);
  const uint32_t* __restrict__ meta = vp(meta_, vs);
  uint2* __restrict__ rl = vp(rl_, vs);
  const unsigned long long* __restrict__ rkm = vp(rkm_, vs);
  const int rows = gd.ty[blockIdx.y];
  extern __shared__ uint32_t cnt[];  // [rows] when NR == 0
  if (meta[3]) return;
  const int lane = threadIdx.x;
  const int chunk = part_chunk(blockIdx.x, nblk);
  uint32_t cr[NR > 0 ? NR : 1];
  if constexpr (NR > 0) {
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      const int t = i * kWave + lane;
      cr[i] = t < rows ? rstart[t] + rhist[(size_t)t * nblk + chunk] : 0u;
    }
  } else {
    for (int t = lane; t < rows; t += kWave) cnt[t] = rstart[t] + rhist[(size_t)t * nblk + chunk];
    __syncthreads();
  }
  __shared__ unsigned long long rk_sh[2 * 2 * kWave];
  if (NR > 0 && rkm) load_row_masks(rk_sh, rkm, rows);
  const int r0 = chunk * kPartRanks;
  // all of the block's entries are loaded before the first is used (one wait for them all;
  // in the scatter a wait for loads issued after stores would also wait for the stores)
  constexpr int kSub = kPartRanks / kWave;
  RectRaw raw[kSub];
#pragma unroll
  for (int q = 0; q < kSub; ++q) raw[q] = part_lane_raw(n, r0 + q * kWave + lane, order, rect);
  // one sub-batch at a time from raw[0], the rest moving down (static register indices)
#pragma unroll 1
  for (int q = 0; q < kSub; ++q) {
    if (r0 + q * kWave >= n) break;
    const RectL l = part_lane_rect(raw[0]);
#pragma unroll
    for (int t = 0; t + 1 < kSub; ++t) raw[t] = raw[t + 1];
    const int y0 = (int)(l.org >> 16), h = l.area / l.w, x0 = (int)(l.org & 0xFFFFu);
    const uint2 e = make_uint2(l.gid, (uint32_t)x0 | ((uint32_t)l.w << 16));
    auto emit = [&](int, uint32_t pos) { rl[pos] = e; };
    if constexpr (NR > 0) {
      // this lane's rows: those of its span, less (with row masks) the rows where the span
      // reaches no wanted tile
      uint64_t u[NR];
#pragma unroll
      for (int i2 = 0; i2 < NR; ++i2) u[i2] = span_bits(y0, h, i2);
      if (rkm) {
        const uint64_t m0 = span_bits(x0, l.w, 0), m1 = span_bits(x0, l.w, 1);
        for (int j = 0; j < h; ++j) {
          const int r = y0 + j;
          if (!row_wanted(rk_sh, r, m0, m1)) {
            if (NR == 1 || r < kWave) u[0] &= ~(1ull << (r & (kWave - 1)));
            else u[NR - 1] &= ~(1ull << (r & (kWave - 1)));
          }
        }
      }
      place_batch_masked<NR>(cr, u, emit);
    } else {
      const int lo = wave_min(h > 0 ? y0 : INT_MAX), hi = wave_max(h > 0 ? y0 + h - 1 : -1);
      const auto all = [](int) { return true; };
      const auto covers = [&](int r) { return h > 0 && y0 <= r && r < y0 + h; };
      place_batch(cnt, lo, hi, lane, emit, all, covers);
    }
  }
}

// ---- level 2: tiles within a row ----------------------------------------------------------
// The level-2 kernels run kWaves2 independent wavefronts per workgroup (more wavefronts per CU
// than one-wave workgroups get); each has its own LDS slice, so a wavefront-level barrier
// orders its LDS accesses.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Chunk ci of the level-2 work: row (binary search over the chunk prefix) and its entries.
struct Chunk2 {
  int row;
  uint32_t begin, end;  // entry range in the row list
  uint32_t idx;         // chunk index within the row
};

// cpl: the block's LDS copy of the chunk prefix.
__device__ __forceinline__ Chunk2 chunk2_of(uint32_t ci, int rows, const uint32_t* cpl,
                                            const uint32_t* __restrict__ rstart, const uint32_t* __restrict__ rtot,
                                            uint32_t K2) {
  int lo = 0, hi = rows - 1;  // last row with cpl[row] <= ci
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (cpl[mid] <= ci) lo = mid; else hi = mid - 1;
  }
  Chunk2 c;
  c.row = lo;
  c.idx = ci - cpl[lo];
  c.begin = rstart[lo] + c.idx * K2;
  c.end = min(c.begin + K2, rstart[lo] + rtot[lo]);
  return c;
}

// Pass 2a: pairs per (tile, chunk); the table of row r holds tiles_x rows of nch[r] chunk
// counts at tiles_x * cp[r]. Persistent: blocks stride over the chunks.
__global__ __launch_bounds__(kWave * kWaves2) void k_tile2_hist(const uint2* rl_, GroupDims gd, const uint32_t* rstart_,
                                                      const uint32_t* rtot_, const uint32_t* cp_, const uint32_t* nch_,
                                                      const uint32_t* meta_, uint32_t* hist2_, size_t vs) {
  const uint2* __restrict__ rl = vp(rl_, vs);
  const uint32_t* __restrict__ rstart = vp(rstart_, vs);
  const uint32_t* __restrict__ rtot = vp(rtot_, vs);
  const uint32_t* __restrict__ cp = vp(cp_, vs);
  const uint32_t* __restrict__ nch = vp(nch_, vs);
  const uint32_t* __restrict__ meta = vp(meta_, vs);
  uint32_t* __restrict__ hist2 = vp(hist2_, vs);
  const int rows = gd.ty[blockIdx.y], tiles_x = gd.tx[blockIdx.y];
  extern __shared__ uint32_t lds2[];  // chunk prefix [rows], then cnt [kWaves2][tiles_x]
  uint32_t* cpl = lds2;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  uint32_t* cnt = lds2 + rows + wave * tiles_x;
  if (meta[3]) return;
  const uint32_t K2 = meta[1], NC = meta[2];
  if (blockIdx.x * kWaves2 >= NC) return;
  for (int r = threadIdx.x; r < rows; r += blockDim.x) cpl[r] = cp[r];
  __syncthreads();
  for (uint32_t ci = blockIdx.x * kWaves2 + wave; ci < NC; ci += gridDim.x * kWaves2) {
    wave_sync();
    const Chunk2 c = chunk2_of(ci, rows, cpl, rstart, rtot, K2);
    for (int t = lane; t < tiles_x; t += kWave) cnt[t] = 0u;
    wave_sync();
    // spans in groups of kGrp batches of 64, all loaded before any is counted (one wait per group)
    constexpr int kGrp = 8;
    for (uint32_t g0 = c.begin; g0 < c.end; g0 += kWave * kGrp) {
      uint32_t xw[kGrp];
#pragma unroll
      for (int q = 0; q < kGrp; ++q) {
        const uint32_t i = g0 + (uint32_t)(q * kWave + lane);
        xw[q] = i < c.end ? rl[i].y : 0u;  // w = 0 past the chunk
      }
#pragma unroll
      for (int q = 0; q < kGrp; ++q) {
        const int x0 = (int)(xw[q] & 0xFFFFu), w = (int)(xw[q] >> 16);
        for (int j = 0; j < w; ++j) atomicAdd(&cnt[x0 + j], 1u);
      }
    }
    wave_sync();
    uint32_t* dst = hist2 + (size_t)tiles_x * cp[c.row];
    const uint32_t nc = nch[c.row];
    for (int t = lane; t < tiles_x; t += kWave) dst[(size_t)t * nc + c.idx] = cnt[t];
  }
}

// Pass 2b: per tile, exclusive scan of its counts across its row's chunks (in place); totals.
__global__ __launch_bounds__(256) void k_tile2_scan(uint32_t* hist2_, GroupDims gd, const uint32_t* cp_,
                                                    const uint32_t* nch_, const uint32_t* meta_, uint32_t* tot_,
                                                    size_t vs) {
  const int tiles_x = gd.tx[blockIdx.y];
  if ((int)blockIdx.x >= tiles_x * gd.ty[blockIdx.y]) return;  // past this view's tiles
  uint32_t* __restrict__ hist2 = vp(hist2_, vs);
  const uint32_t* __restrict__ cp = vp(cp_, vs);
  const uint32_t* __restrict__ nch = vp(nch_, vs);
  const uint32_t* __restrict__ meta = vp(meta_, vs);
  uint32_t* __restrict__ tot = vp(tot_, vs);
  __shared__ uint32_t sm[256];
  const int tile = blockIdx.x;
  const int r = tile / tiles_x, x = tile % tiles_x;
  const int nc = meta[3] ? 0 : (int)nch[r];
  uint32_t* row = hist2 + (size_t)tiles_x * cp[r] + (size_t)x * nc;
  uint32_t carry = 0;
  for (int b0 = 0; b0 < nc; b0 += 256) {
    const int i = b0 + threadIdx.x;
    const uint32_t v = (i < nc) ? row[i] : 0u;
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
      const uint32_t add = (threadIdx.x >= (unsigned)off) ? sm[threadIdx.x - off] : 0u;
      __syncthreads();
      sm[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nc) row[i] = carry + sm[threadIdx.x] - v;
    carry += sm[255];
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[tile] = carry;
}

// Pass 2c: each chunk's entries, in order, to their tiles: ranges[tile] + (pairs of earlier
// chunks of the row for the tile) + (earlier pairs of this chunk). Entries of a row are in
// depth order and the placement keeps lane order within a tile: stable. A block keeps at most
// tiles_x output runs open, so the L2 completes their lines. NR > 0: counters in registers
// (tiles_x <= 64 NR) and only the covered, wanted tiles visited; else counters in LDS.
template <int NR>
__global__ __launch_bounds__(kWave * kWaves2) void k_tile2_scatter(const uint2* rl_, GroupDims gd, const uint32_t* rstart_,
                                                         const uint32_t* rtot_, const uint32_t* cp_,
                                                         const uint32_t* nch_, const uint32_t* meta_,
                                                         const uint32_t* hist2_, const uint32_t* ranges_,
                                                         int64_t capacity, uint32_t* gids_out_, const int32_t* keep_,
                                                         size_t vs) {
  const uint2* __restrict__ rl = vp(rl_, vs);
  const uint32_t* __restrict__ rstart = vp(rstart_, vs);
  const uint32_t* __restrict__ rtot = vp(rtot_, vs);
  const uint32_t* __restrict__ cp = vp(cp_, vs);
  const uint32_t* __restrict__ nch = vp(nch_, vs);
  const uint32_t* __restrict__ meta = vp(meta_, vs);
  const uint32_t* __restrict__ hist2 = vp(hist2_, vs);
  const uint32_t* __restrict__ ranges = vp(ranges_, vs);
  uint32_t* __restrict__ gids_out = vp(gids_out_, vs);
  const int32_t* __restrict__ keep = vp(keep_, vs);
  const int rows = gd.ty[blockIdx.y], tiles_x = gd.tx[blockIdx.y];
  extern __shared__ uint32_t lds2[];  // chunk prefix [rows], then (NR == 0) cnt [kWaves2][tiles_x]
  uint32_t* cpl = lds2;
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  uint32_t* cnt = lds2 + rows + wave * tiles_x;
  if (meta[3]) return;
  const uint32_t K2 = meta[1], NC = meta[2];
  // positions stay below M <= capacity here (a view whose M exceeds the capacity returned
  // above); the clamp below only keeps a stray position inside the list buffer, without a
  // branch per store
  const uint32_t cap_last = (uint32_t)min(max(capacity, (int64_t)1) - 1, (int64_t)0xFFFFFFFF);
  if (blockIdx.x * kWaves2 >= NC) return;
  for (int r = threadIdx.x; r < rows; r += blockDim.x) cpl[r] = cp[r];
  __syncthreads();
  for (uint32_t ci = blockIdx.x * kWaves2 + wave; ci < NC; ci += gridDim.x * kWaves2) {
    wave_sync();
    const Chunk2 c = chunk2_of(ci, rows, cpl, rstart, rtot, K2);
    const uint32_t* h = hist2 + (size_t)tiles_x * cp[c.row];
    const uint32_t nc = nch[c.row];
    const int tbase = c.row * tiles_x;
    uint32_t cr[NR > 0 ? NR : 1];
    uint64_t km[NR > 0 ? NR : 1];  // wanted tiles of the row, bit t % 64 of word t / 64
    if constexpr (NR > 0) {
#pragma unroll
      for (int i2 = 0; i2 < NR; ++i2) {
        const int t = i2 * kWave + lane;
        cr[i2] = t < tiles_x ? ranges[tbase + t] + h[(size_t)t * nc + c.idx] : 0u;
        km[i2] = __ballot(t < tiles_x && (!keep || keep[tbase + t] != 0));
      }
    } else {
      for (int t = lane; t < tiles_x; t += kWave) cnt[t] = ranges[tbase + t] + h[(size_t)t * nc + c.idx];
      wave_sync();
    }
    // Entries go in groups of kGrp batches of 64, the next group's loaded while the current one
    // is placed: a wait for loads (which also waits for the stores before it) comes once per
    // group, not once per batch. Entries past the chunk have w = 0 and cover nothing.
    constexpr int kGrp = 8;
    uint2 cur[kGrp], nxt[kGrp];
#pragma unroll
    for (int q = 0; q < kGrp; ++q) {
      const uint32_t i = c.begin + (uint32_t)(q * kWave + lane);
      cur[q] = i < c.end ? rl[i] : make_uint2(0u, 0u);
    }
    for (uint32_t g0 = c.begin; g0 < c.end; g0 += kWave * kGrp) {
      // every entry of the group in registers before the next group's loads are issued (the
      // empty asm consumes them, and its memory clobber keeps those loads behind it)
      uint32_t any = 0u;
#pragma unroll
      for (int q = 0; q < kGrp; ++q) any |= cur[q].x | cur[q].y;
      asm volatile("" ::"v"(any) : "memory");
#pragma unroll
      for (int q = 0; q < kGrp; ++q) {
        const uint32_t i = g0 + (uint32_t)((kGrp + q) * kWave + lane);
        nxt[q] = i < c.end ? rl[i] : make_uint2(0u, 0u);
      }
      // one batch at a time from cur[0], the rest moving down (static register indices)
#pragma unroll 1
      for (int q = 0; q < kGrp; ++q) {
      if (g0 + (uint32_t)(q * kWave) >= c.end) break;
      const uint2 e = cur[0];
#pragma unroll
      for (int t = 0; t + 1 < kGrp; ++t) cur[t] = cur[t + 1];
      const int x0 = (int)(e.y & 0xFFFFu), w = (int)(e.y >> 16);
      auto emit = [&](int, uint32_t pos) {
        gids_out[min(pos, cap_last)] = e.x;
      };
      if constexpr (NR > 0) {
        uint64_t u[NR];
#pragma unroll
        for (int i2 = 0; i2 < NR; ++i2) u[i2] = span_bits(x0, w, i2) & km[i2];
        place_batch_masked<NR>(cr, u, emit);
      } else {
        const int lo = wave_min(w > 0 ? x0 : INT_MAX), hi = wave_max(w > 0 ? x0 + w - 1 : -1);
        const auto kept = [&](int t) { return !keep || keep[tbase + t] != 0; };
        const auto covers = [&](int t) { return w > 0 && x0 <= t && t < x0 + w; };
        place_batch(cnt, lo, hi, lane, emit, kept, covers);
      }
      }
#pragma unroll
      for (int q = 0; q < kGrp; ++q) cur[q] = nxt[q];
    }
  }
}

// keys (tile << 32 | depth bits) of the sorted pairs: one block per tile.
__global__ __launch_bounds__(256) void k_keys64(const uint32_t* __restrict__ ranges, int ntiles,
                                                const uint32_t* __restrict__ gids, const uint32_t* __restrict__ zkey,
                                                uint64_t* __restrict__ keys) {
  const uint32_t t = blockIdx.x;
  for (uint32_t i = ranges[t] + threadIdx.x; i < ranges[ntiles + t]; i += blockDim.x)
    keys[i] = ((uint64_t)t << 32) | (uint64_t)zkey[gids[i]];
}

}  // namespace

// Workspace layout (all 256-byte aligned):
//   dkeys[2], dvals[2]: u32 [n]          depth-sort ping-pong
//   m_total: u64 [1], blocksum: u64 [ceil(n / 4096) + 1]
//   phist: u32 [4096][ceil(n / 256)]     pairs per (tile, partition block)
//   ptot: u32 [4096]
//   hist: u32 [256][blocks(n)], rowtot: u32 [256]   radix-sort scratch
size_t bin_ws_bytes(int64_t n, int64_t max_pairs) {
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  const size_t nb = sort_blocks_for(nn);
  const size_t nblk = (nn + kPartRanks - 1) / kPartRanks;
  const size_t mp = (size_t)std::max<int64_t>(max_pairs, 1);
  size_t b = 0;
  b += 4 * align_up(nn * 4, 256);
  b += align_up(8, 256);
  b += align_up(((nn + kScanTile - 1) / kScanTile + 1) * 8, 256);
  b += align_up((size_t)NGS_MAX_TILES * nblk * 4, 256);
  b += align_up((size_t)NGS_MAX_TILES * 4, 256);
  b += align_up(256 * nb * 4, 256);
  b += align_up(256 * 4, 256);
  b += align_up(mp * 8, 256);                          // row entries
  b += align_up(nn * 8, 256);                          // rects in depth order
  b += align_up((size_t)kHist2 * 4, 256);              // level-2 counts
  b += 4 * align_up(((size_t)NGS_MAX_TILES + 1) * 4, 256);  // rtot, rstart, nch, cp
  b += align_up(16, 256);                              // meta
  b += align_up((size_t)NGS_MAX_TILES * 16, 256);      // wanted-tile masks per row
  return b;
}

BinWs bin_ws_carve(void* ws, int64_t n, int64_t max_pairs) {
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  const size_t nb = sort_blocks_for(nn);
  const size_t nblk = (nn + kPartRanks - 1) / kPartRanks;
  const size_t mp = (size_t)std::max<int64_t>(max_pairs, 1);
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t bytes) { char* r = p; p += align_up(bytes, 256); return r; };
  BinWs w;
  for (int i = 0; i < 2; ++i) w.dkeys[i] = (uint32_t*)take(nn * 4);
  for (int i = 0; i < 2; ++i) w.dvals[i] = (uint32_t*)take(nn * 4);
  w.m_total = (uint64_t*)take(8);
  w.blocksum = (uint64_t*)take(((nn + kScanTile - 1) / kScanTile + 1) * 8);
  w.phist = (uint32_t*)take((size_t)NGS_MAX_TILES * nblk * 4);
  w.ptot = (uint32_t*)take((size_t)NGS_MAX_TILES * 4);
  w.sort.hist = (uint32_t*)take(256 * nb * 4);
  w.sort.rowtot = (uint32_t*)take(256 * 4);
  w.sort.max_blocks = nb;
  w.rl = (uint2*)take(mp * 8);
  w.rect_sorted = (int16_t*)take(nn * 8);
  w.hist2 = (uint32_t*)take((size_t)kHist2 * 4);
  w.rtot = (uint32_t*)take(((size_t)NGS_MAX_TILES + 1) * 4);
  w.rstart = (uint32_t*)take(((size_t)NGS_MAX_TILES + 1) * 4);
  w.nch = (uint32_t*)take(((size_t)NGS_MAX_TILES + 1) * 4);
  w.cp = (uint32_t*)take(((size_t)NGS_MAX_TILES + 1) * 4);
  w.meta = (uint32_t*)take(16);
  w.rkm = (unsigned long long*)take((size_t)NGS_MAX_TILES * 16);
  return w;
}

// Depth sort of all n Gaussians (culled ones carry key 0xFFFFFFFF and sort last) and the
// view's pair count M (*m_total).
hipError_t bin_count_pairs(const ngs_projected& p, int n, const BinWs& w, hipStream_t st, int g, size_t vs) {
  uint32_t *ko, *vo;
  // inputs: zkey (read only), values = gids (implicit); ping-pong (dkeys[0], dvals[0]) / (dkeys[1], dvals[1])
  hipError_t e = radix_sort_pairs(p.zkey, nullptr, w.dkeys[0], w.dvals[0], w.dkeys[1], w.dvals[1], (size_t)n, 0, 32,
                                  w.sort, st, &ko, &vo, kProfDepthHist, p.rect, w.rect_sorted, g, vs);
  if (e != hipSuccess) return e;
  // 4 passes: result in (dkeys[1], dvals[1])
  const int nb = (n + kScanTile - 1) / kScanTile;
  if (n > 0) {
    ProfScope ps(kProfCountScan, st);
    hipLaunchKernelGGL(k_count_partials, dim3(nb, g), dim3(kScanThreads), 0, st, p.count, n, w.blocksum, vs);
    hipLaunchKernelGGL(k_count_total, dim3(1, g), dim3(kScanThreads), 0, st, w.blocksum, nb, w.m_total, vs);
  } else {
    e = launch_fill_u32(reinterpret_cast<uint32_t*>(w.m_total), 0u, 2, st, g, vs);
  }
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t bin_emit_and_sort(const ngs_projected& p, int n, const Group& G, const BinWs& w,
                             const ngs_tile_lists& out, int32_t* overflow, int64_t* stats, hipStream_t st,
                             const int32_t* keep, int chunk2) {
  const int g = G.g;
  const size_t vs = G.vs;
  const int rows = G.max_tiles_y, tx = G.max_tiles_x, ntiles = G.max_ntiles;  // largest view of the group
  const uint32_t* order = w.dvals[1];
  const uint64_t* m_total = w.m_total;
  if (n == 0) {
    hipError_t e = launch_fill_u32(reinterpret_cast<uint32_t*>(out.n_pairs), 0u, 2, st, g, vs);
    return e != hipSuccess ? e : launch_fill_u32(out.ranges, 0u, 2 * (size_t)ntiles, st, g, vs);
  }
  const int nblk = (n + kPartRanks - 1) / kPartRanks;
  const int grid2 = std::max(256, kGrid2 / g) / kWaves2;  // persistent level-2 workgroups per view
  const unsigned long long* rkm = nullptr;
  if (keep && tx <= 2 * kWave && rows <= 2 * kWave) {
    ProfScope ps(kProfTileHist, st);
    hipLaunchKernelGGL(k_keep_rows, dim3(1, g), dim3(256), 0, st, keep, G.dims, w.rkm, vs);
    rkm = w.rkm;
  }
  {
    ProfScope ps(kProfTileHist, st);
    hipLaunchKernelGGL(k_row_hist, dim3(nblk, g), dim3(kWave), rows * 4, st, n, order, w.rect_sorted, G.dims, w.phist,
                       nblk, rkm, vs);
  }
  {
    ProfScope ps(kProfTileScan, st);
    hipLaunchKernelGGL(k_part_scan_rows, dim3(rows, g), dim3(256), 0, st, w.phist, nblk, w.rtot, G.dims, vs);
    hipLaunchKernelGGL(k_row_starts, dim3(1, g), dim3(256), 0, st, w.rtot, G.dims, m_total, out.capacity, w.rstart,
                       w.nch, w.cp, w.meta, out.n_pairs, (uint32_t)(chunk2 > 0 ? chunk2 : kChunk2), vs);
  }
  {
    ProfScope ps(kProfTileScatter, st);
    if (rows <= kWave)
      hipLaunchKernelGGL(k_row_scatter<1>, dim3(nblk, g), dim3(kWave), 0, st, n, order, w.rect_sorted, G.dims, w.phist,
                         nblk, w.rstart, w.meta, w.rl, rkm, vs);
    else if (rows <= 2 * kWave)
      hipLaunchKernelGGL(k_row_scatter<2>, dim3(nblk, g), dim3(kWave), 0, st, n, order, w.rect_sorted, G.dims, w.phist,
                         nblk, w.rstart, w.meta, w.rl, rkm, vs);
    else
      hipLaunchKernelGGL(k_row_scatter<0>, dim3(nblk, g), dim3(kWave), rows * 4, st, n, order, w.rect_sorted, G.dims,
                         w.phist, nblk, w.rstart, w.meta, w.rl, rkm, vs);
  }
  {
    ProfScope ps(kProfTileHist, st);
    hipLaunchKernelGGL(k_tile2_hist, dim3(grid2, g), dim3(kWave * kWaves2), (kWaves2 * tx + rows) * 4, st, w.rl, G.dims,
                       w.rstart, w.rtot,
                       w.cp, w.nch, w.meta, w.hist2, vs);
  }
  {
    ProfScope ps(kProfTileScan, st);
    hipLaunchKernelGGL(k_tile2_scan, dim3(ntiles, g), dim3(256), 0, st, w.hist2, G.dims, w.cp, w.nch, w.meta, w.ptot,
                       vs);
    hipLaunchKernelGGL(k_part_ranges, dim3(1, g), dim3(256), 0, st, w.ptot, G.dims, out.ranges, out.capacity, overflow,
                       stats, m_total, keep, vs);
  }
  {
    ProfScope ps(kProfTileScatter, st);
    if (tx <= kWave)
      hipLaunchKernelGGL(k_tile2_scatter<1>, dim3(grid2, g), dim3(kWave * kWaves2), rows * 4, st, w.rl, G.dims, w.rstart,
                         w.rtot, w.cp, w.nch, w.meta, w.hist2, out.ranges, out.capacity, out.gids, keep, vs);
    else if (tx <= 2 * kWave)
      hipLaunchKernelGGL(k_tile2_scatter<2>, dim3(grid2, g), dim3(kWave * kWaves2), rows * 4, st, w.rl, G.dims, w.rstart,
                         w.rtot, w.cp, w.nch, w.meta, w.hist2, out.ranges, out.capacity, out.gids, keep, vs);
    else
      hipLaunchKernelGGL(k_tile2_scatter<0>, dim3(grid2, g), dim3(kWave * kWaves2), (kWaves2 * tx + rows) * 4, st, w.rl,
                         G.dims,
                         w.rstart, w.rtot, w.cp, w.nch, w.meta, w.hist2, out.ranges, out.capacity, out.gids, keep, vs);
  }
  if (out.keys && g == 1) {
    ProfScope ps(kProfKeys64, st);
    hipLaunchKernelGGL(k_keys64, dim3(ntiles), dim3(256), 0, st, out.ranges, ntiles, out.gids, p.zkey, out.keys);
  }
  return hipGetLastError();
}

}  // namespace ngs
