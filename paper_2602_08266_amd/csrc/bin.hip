// bin.hip -- tile binning: (tile, depth, gid)-sorted lists of every (tile, Gaussian) pair.
//
// The sort is an LSD radix sort on the composite key (tile, float32 depth bits, gid) run in
// two stages, because all pairs of one Gaussian share its depth bits:
//   1. depth digits: the n Gaussians are sorted by their 32-bit depth key (4 passes over n
//      entries instead of over the M >> n pairs); gid order breaks ties (stable LSD);
//   2. one stable counting pass on the tile digit (<= 12 bits) over the pairs, fused with
//      their generation: each single-wavefront block takes 512 consecutive depth ranks one
//      Gaussian at a time (its lanes spread over that Gaussian's rect), counts its pairs per
//      tile (pass a), and after a scan over blocks and tiles (pass b) writes each pair's gid
//      at its final position (pass c); per-tile positions advance in depth order.
// The result equals a sort of (tile << 32 | depth bits) with ties broken by gid; the
// per-tile ranges fall out of the scan, and no pair array other than the output is written.
#include "common.hpp"

namespace ngs {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Exclusive scan (u64) of count[gid_sorted[i]]: per-block local scan and block totals.
__global__ __launch_bounds__(kScanThreads) void k_scan_local(const uint32_t* __restrict__ count,
                                                             const uint32_t* __restrict__ order, int n,
                                                             uint64_t* __restrict__ out, uint64_t* __restrict__ bsum) {
  __shared__ uint64_t sm[kScanThreads];
  const int t = threadIdx.x;
  const int base = blockIdx.x * kScanTile + t * kScanItems;
  uint64_t v[kScanItems];
  uint64_t run = 0;
  for (int j = 0; j < kScanItems; ++j) {
    const int i = base + j;
    const uint64_t c = (i < n) ? (uint64_t)count[order[i]] : 0ull;
    v[j] = run;
    run += c;
  }
  sm[t] = run;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint64_t add = (t >= off) ? sm[t - off] : 0ull;
    __syncthreads();
    sm[t] += add;
    __syncthreads();
  }
  const uint64_t excl = sm[t] - run;
  for (int j = 0; j < kScanItems; ++j)
    if (base + j < n) out[base + j] = excl + v[j];
  if (t == kScanThreads - 1) bsum[blockIdx.x] = sm[t];
}

// Single block: exclusive scan of the block totals in place; writes the grand total.
__global__ __launch_bounds__(kScanThreads) void k_scan_blocks(uint64_t* __restrict__ bsum, int nb,
                                                              uint64_t* __restrict__ total) {
  __shared__ uint64_t sm[kScanThreads];
  const int t = threadIdx.x;
  uint64_t carry = 0;
  for (int b0 = 0; b0 < nb; b0 += kScanThreads) {
    const int i = b0 + t;
    const uint64_t v = (i < nb) ? bsum[i] : 0ull;
    sm[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
      const uint64_t add = (t >= off) ? sm[t - off] : 0ull;
      __syncthreads();
      sm[t] += add;
      __syncthreads();
    }
    if (i < nb) bsum[i] = carry + sm[t] - v;
    carry += sm[kScanThreads - 1];
    __syncthreads();
  }
  if (t == 0) *total = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(uint64_t* __restrict__ out, int n,
                                                           const uint64_t* __restrict__ bsum) {
  const int i = blockIdx.x * kScanTile + threadIdx.x;
  const uint64_t add = bsum[blockIdx.x];
  for (int j = 0; j < kScanItems; ++j) {
    const int ii = i + j * kScanThreads;
    if (ii < n) out[ii] += add;
  }
}

constexpr int kPartRanks = 512;  // depth ranks per partition block (one wavefront)

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

__device__ __forceinline__ RectL part_lane_load(int n, int r, const uint32_t* __restrict__ order,
                                                const int16_t* __restrict__ rect) {
  RectL l{0u, 0u, 1, 0, 1.f};
  if (r < n) {
    const uint32_t g = order[r];
    const short4 b = reinterpret_cast<const short4*>(rect)[g];
    l.gid = g;
    l.org = (uint32_t)(uint16_t)b.x | ((uint32_t)(uint16_t)b.y << 16);
    l.w = b.z - b.x + 1;
    l.area = b.z >= b.x ? l.w * (b.w - b.y + 1) : 0;
    l.w = l.area > 0 ? l.w : 1;
    l.inv_w = 1.f / (float)l.w;
  }
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

// Pass a: pairs per (tile, block), tile-major: hist[t * nblk + block]. Each lane loads one
// Gaussian of the current 64 ranks; the wavefront then takes them one at a time (values
// broadcast from that lane) and spreads its lanes over the Gaussian's tiles, which are
// distinct, adding to the per-tile counters with LDS atomics.
__global__ __launch_bounds__(kWave) void k_part_hist(int n, const uint32_t* __restrict__ order,
                                                     const int16_t* __restrict__ rect, int tiles_x, int ntiles,
                                                     uint32_t* __restrict__ hist, int nblk) {
  __shared__ uint32_t cnt[NGS_MAX_TILES];
  const int lane = threadIdx.x;
  const int chunk = part_chunk(blockIdx.x, nblk);
  for (int t = lane; t < ntiles; t += kWave) cnt[t] = 0u;
  __syncthreads();
  const int r0 = chunk * kPartRanks;
  for (int sub = 0; sub < kPartRanks && r0 + sub < n; sub += kWave) {
    const RectL l = part_lane_load(n, r0 + sub + lane, order, rect);
    for (int q = 0; q < kWave; ++q) {
      const RectU u = part_bcast(l, q);
      for (int j = lane; j < u.area; j += kWave) atomicAdd(&cnt[part_tile(u, j, tiles_x)], 1u);
    }
  }
  __syncthreads();
  for (int t = lane; t < ntiles; t += kWave) hist[(size_t)t * nblk + chunk] = cnt[t];
}

// Pass b1: per tile, exclusive scan of its counts across blocks (in place); totals.
__global__ __launch_bounds__(256) void k_part_scan_rows(uint32_t* __restrict__ hist, int nblk,
                                                        uint32_t* __restrict__ tot) {
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

// Pass b2: tile starts (exclusive scan of the totals) -> ranges; an empty tile gets
// start = end = the number of pairs in lower tiles. If the pairs exceed the list capacity,
// every range is left empty and *overflow is raised (the scatter then writes nothing).
__global__ __launch_bounds__(256) void k_part_ranges(const uint32_t* __restrict__ tot, int ntiles,
                                                     uint32_t* __restrict__ ranges, int64_t capacity,
                                                     int32_t* __restrict__ overflow, int64_t* __restrict__ stats) {
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
  const uint32_t total = sm[255];
  const bool over = (int64_t)total > capacity;
  const uint32_t excl = sm[threadIdx.x] - run;
  for (int j = 0; j < kPer; ++j)
    if (t0 + j < ntiles) {
      ranges[t0 + j] = over ? 0u : excl + v[j];
      ranges[ntiles + t0 + j] = over ? 0u : excl + v[j] + tot[t0 + j];
    }
  if (threadIdx.x == 0) {
    if (over && overflow) atomicOr(overflow, 1);
    if (stats) atomicAdd((unsigned long long*)&stats[1], (unsigned long long)total);
  }
}

// Pass c: every pair goes to ranges[tile] + (pairs of lower blocks for the tile) + (earlier
// pairs of this block for the tile). The wavefront takes its Gaussians one at a time in
// depth order and its LDS atomics execute in program order, so each tile's running
// position advances in depth order: the pass is stable.
__global__ __launch_bounds__(kWave) void k_part_scatter(int n, const uint32_t* __restrict__ order,
                                                        const int16_t* __restrict__ rect, int tiles_x, int ntiles,
                                                        const uint32_t* __restrict__ hist, int nblk,
                                                        const uint32_t* __restrict__ ranges, int64_t capacity,
                                                        uint32_t* __restrict__ gids_out) {
  __shared__ uint32_t cnt[NGS_MAX_TILES];
  const int lane = threadIdx.x;
  const int chunk = part_chunk(blockIdx.x, nblk);
  for (int t = lane; t < ntiles; t += kWave) cnt[t] = ranges[t] + hist[(size_t)t * nblk + chunk];
  __syncthreads();
  const int r0 = chunk * kPartRanks;
  for (int sub = 0; sub < kPartRanks && r0 + sub < n; sub += kWave) {
    const RectL l = part_lane_load(n, r0 + sub + lane, order, rect);
    for (int q = 0; q < kWave; ++q) {
      const RectU u = part_bcast(l, q);
      for (int j = lane; j < u.area; j += kWave) {
        const uint32_t pos = atomicAdd(&cnt[part_tile(u, j, tiles_x)], 1u);
        if ((int64_t)pos < capacity) gids_out[pos] = u.gid;
      }
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
//   offsets: u64 [n + 1], blocksum: u64 [ceil(n / 1024) + 1]
//   phist: u32 [4096][ceil(n / 256)]     pairs per (tile, partition block)
//   ptot: u32 [4096]
//   hist: u32 [256][blocks(n)], rowtot: u32 [256]   radix-sort scratch
size_t bin_ws_bytes(int64_t n, int64_t max_pairs) {
  (void)max_pairs;
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  const size_t nb = sort_blocks_for(nn);
  const size_t nblk = (nn + kPartRanks - 1) / kPartRanks;
  size_t b = 0;
  b += 4 * align_up(nn * 4, 256);
  b += align_up((nn + 1) * 8, 256);
  b += align_up(((nn + kScanTile - 1) / kScanTile + 1) * 8, 256);
  b += align_up((size_t)NGS_MAX_TILES * nblk * 4, 256);
  b += align_up((size_t)NGS_MAX_TILES * 4, 256);
  b += align_up(256 * nb * 4, 256);
  b += align_up(256 * 4, 256);
  return b;
}

BinWs bin_ws_carve(void* ws, int64_t n, int64_t max_pairs) {
  (void)max_pairs;
  const size_t nn = (size_t)std::max<int64_t>(n, 1);
  const size_t nb = sort_blocks_for(nn);
  const size_t nblk = (nn + kPartRanks - 1) / kPartRanks;
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t bytes) { char* r = p; p += align_up(bytes, 256); return r; };
  BinWs w;
  for (int i = 0; i < 2; ++i) w.dkeys[i] = (uint32_t*)take(nn * 4);
  for (int i = 0; i < 2; ++i) w.dvals[i] = (uint32_t*)take(nn * 4);
  w.offsets = (uint64_t*)take((nn + 1) * 8);
  w.blocksum = (uint64_t*)take(((nn + kScanTile - 1) / kScanTile + 1) * 8);
  w.phist = (uint32_t*)take((size_t)NGS_MAX_TILES * nblk * 4);
  w.ptot = (uint32_t*)take((size_t)NGS_MAX_TILES * 4);
  w.sort.hist = (uint32_t*)take(256 * nb * 4);
  w.sort.rowtot = (uint32_t*)take(256 * 4);
  w.sort.max_blocks = nb;
  return w;
}

// Depth sort of all n Gaussians (culled ones carry key 0xFFFFFFFF and sort last) and the
// exclusive scan of their tile counts in that order; offsets[n] = M.
hipError_t bin_count_pairs(const ngs_projected& p, int n, const BinWs& w, hipStream_t st) {
  hipError_t e = launch_iota(w.dvals[1], (size_t)n, st);
  if (e != hipSuccess) return e;
  uint32_t *ko, *vo;
  // inputs: zkey (read only) and iota in dvals[1]; ping-pong (dkeys[0], dvals[0]) / (dkeys[1], dvals[1])
  e = radix_sort_pairs(p.zkey, w.dvals[1], w.dkeys[0], w.dvals[0], w.dkeys[1], w.dvals[1], (size_t)n, 0, 32,
                       w.sort, st, &ko, &vo, kProfDepthHist);
  if (e != hipSuccess) return e;
  // 4 passes: result in (dkeys[1], dvals[1])
  const int nb = (n + kScanTile - 1) / kScanTile;
  if (n > 0) {
    ProfScope ps(kProfCountScan, st);
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(kScanThreads), 0, st, p.count, vo, n, w.offsets, w.blocksum);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(kScanThreads), 0, st, w.blocksum, nb, w.offsets + n);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanThreads), 0, st, w.offsets, n, w.blocksum);
  } else {
    e = launch_fill_u32(reinterpret_cast<uint32_t*>(w.offsets), 0u, 2, st);
  }
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t bin_emit_and_sort(const ngs_projected& p, int n, const DevCam& cam, const BinWs& w,
                             const ngs_tile_lists& out, int32_t* overflow, int64_t* stats, hipStream_t st) {
  const int ntiles = cam.tiles_x * cam.tiles_y;
  const uint32_t* order = w.dvals[1];
  hipError_t e = launch_copy_u32(reinterpret_cast<uint32_t*>(out.n_pairs),
                                 reinterpret_cast<const uint32_t*>(w.offsets + n), 2, st);
  if (e != hipSuccess) return e;
  if (n == 0) return launch_fill_u32(out.ranges, 0u, 2 * (size_t)ntiles, st);
  const int nblk = (n + kPartRanks - 1) / kPartRanks;
  {
    ProfScope ps(kProfTileHist, st);
    hipLaunchKernelGGL(k_part_hist, dim3(nblk), dim3(kWave), 0, st, n, order, p.rect, cam.tiles_x, ntiles, w.phist,
                       nblk);
  }
  {
    ProfScope ps(kProfTileScan, st);
    hipLaunchKernelGGL(k_part_scan_rows, dim3(ntiles), dim3(256), 0, st, w.phist, nblk, w.ptot);
    hipLaunchKernelGGL(k_part_ranges, dim3(1), dim3(256), 0, st, w.ptot, ntiles, out.ranges, out.capacity, overflow,
                       stats);
  }
  {
    ProfScope ps(kProfTileScatter, st);
    hipLaunchKernelGGL(k_part_scatter, dim3(nblk), dim3(kWave), 0, st, n, order, p.rect, cam.tiles_x, ntiles,
                       w.phist, nblk, out.ranges, out.capacity, out.gids);
  }
  if (out.keys) {
    ProfScope ps(kProfKeys64, st);
    hipLaunchKernelGGL(k_keys64, dim3(ntiles), dim3(256), 0, st, out.ranges, ntiles, out.gids, p.zkey, out.keys);
  }
  return hipGetLastError();
}

}  // namespace ngs
