// bin.hip -- tile binning: (tile, depth, gid)-sorted lists of every (tile, Gaussian) pair.
//
// The sort is an LSD radix sort on the composite key (tile, float32 depth bits, gid) run in
// two stages, because all pairs of one Gaussian share its depth bits:
//   1. depth digits: the n Gaussians are sorted by their 32-bit depth key (4 passes over n
//      entries instead of over the M >> n pairs); gid order breaks ties (stable LSD);
//   2. the pairs are emitted in that depth order and a stable pass on the tile digits
//      (ceil(log2 tiles) bits) groups them by tile without disturbing the depth order.
// The result equals a sort of (tile << 32 | depth bits) with ties broken by gid.
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

// Emission in depth order. A block owns 256 consecutive depth ranks and the contiguous
// output range [offsets[r0], offsets[r0 + 256]); its lanes stride over that range, so the
// writes are coalesced and a Gaussian with a huge rect is expanded by the whole block. Each
// output finds its Gaussian by binary search over the block's offsets in LDS; a Gaussian's
// tiles go row by row.
constexpr int kEmitRanks = 256;

__global__ __launch_bounds__(kEmitRanks) void k_emit(int n, const uint32_t* __restrict__ order,
                                                     const uint64_t* __restrict__ offsets,
                                                     const int16_t* __restrict__ rect, int tiles_x,
                                                     uint32_t* __restrict__ tkey, uint32_t* __restrict__ tval) {
  __shared__ uint64_t s_off[kEmitRanks + 1];
  __shared__ uint32_t s_gid[kEmitRanks];
  __shared__ int32_t s_x0[kEmitRanks], s_y0[kEmitRanks], s_w[kEmitRanks];
  const int r0 = blockIdx.x * kEmitRanks;
  const int cnt = min(kEmitRanks, n - r0);
  const int t = threadIdx.x;
  if (t < cnt) {
    const uint32_t g = order[r0 + t];
    s_gid[t] = g;
    s_x0[t] = rect[g];
    s_y0[t] = rect[n + g];
    s_w[t] = rect[2 * n + g] - rect[g] + 1;
    s_off[t] = offsets[r0 + t];
  }
  if (t == 0) s_off[cnt] = offsets[r0 + cnt];
  __syncthreads();
  const uint64_t beg = s_off[0], end = s_off[cnt];
  for (uint64_t p = beg + t; p < end; p += kEmitRanks) {
    // largest i with s_off[i] <= p (entries with zero tiles are skipped by the search)
    int lo = 0, hi = cnt;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (s_off[mid] <= p) lo = mid; else hi = mid;
    }
    const uint32_t j = (uint32_t)(p - s_off[lo]);
    const uint32_t w = (uint32_t)s_w[lo];
    const uint32_t ty = (uint32_t)s_y0[lo] + j / w, tx = (uint32_t)s_x0[lo] + j % w;
    tkey[p] = ty * (uint32_t)tiles_x + tx;
    tval[p] = s_gid[lo];
  }
}

// Per-tile [start, end) over the tile-sorted pairs. An empty tile gets start = end = the
// number of pairs in lower tiles; each gap between two present tiles is filled by the
// thread that sees the second one.
__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ tkey, int64_t m,
                                                uint32_t* __restrict__ ranges, int ntiles) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const uint32_t t = tkey[i];
  if (i == 0 || tkey[i - 1] != t) {
    ranges[t] = (uint32_t)i;
    const uint32_t prev = (i == 0) ? 0u : tkey[i - 1] + 1u;
    for (uint32_t u = prev; u < t; ++u) { ranges[u] = (uint32_t)i; ranges[ntiles + u] = (uint32_t)i; }
  }
  if (i == m - 1 || tkey[i + 1] != t) {
    ranges[ntiles + t] = (uint32_t)(i + 1);
    if (i == m - 1)
      for (int u = (int)t + 1; u < ntiles; ++u) { ranges[u] = (uint32_t)m; ranges[ntiles + u] = (uint32_t)m; }
  }
}

__global__ __launch_bounds__(256) void k_keys64(const uint32_t* __restrict__ tkey, const uint32_t* __restrict__ gids,
                                                const uint32_t* __restrict__ zkey, int64_t m,
                                                uint64_t* __restrict__ keys) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  keys[i] = ((uint64_t)tkey[i] << 32) | (uint64_t)zkey[gids[i]];
}

}  // namespace

// Workspace layout (all 256-byte aligned):
//   dkeys[2], dvals[2]: u32 [n]        depth-sort ping-pong
//   offsets: u64 [n + 1], blocksum: u64 [ceil(n / 1024)]
//   tkeys[2]: u32 [max_pairs], tvals: u32 [max_pairs]
//   hist: u32 [256][blocks(max(n, max_pairs))], rowtot: u32 [256]
size_t bin_ws_bytes(int64_t n, int64_t max_pairs) {
  const size_t nn = (size_t)std::max<int64_t>(n, 1), mp = (size_t)std::max<int64_t>(max_pairs, 1);
  const size_t nb = sort_blocks_for(std::max(nn, mp));
  size_t b = 0;
  b += 4 * align_up(nn * 4, 256);
  b += align_up((nn + 1) * 8, 256);
  b += align_up(((nn + kScanTile - 1) / kScanTile + 1) * 8, 256);
  b += 3 * align_up(mp * 4, 256);
  b += align_up(256 * nb * 4, 256);
  b += align_up(256 * 4, 256);
  return b;
}

BinWs bin_ws_carve(void* ws, int64_t n, int64_t max_pairs) {
  const size_t nn = (size_t)std::max<int64_t>(n, 1), mp = (size_t)std::max<int64_t>(max_pairs, 1);
  const size_t nb = sort_blocks_for(std::max(nn, mp));
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t bytes) { char* r = p; p += align_up(bytes, 256); return r; };
  BinWs w;
  for (int i = 0; i < 2; ++i) w.dkeys[i] = (uint32_t*)take(nn * 4);
  for (int i = 0; i < 2; ++i) w.dvals[i] = (uint32_t*)take(nn * 4);
  w.offsets = (uint64_t*)take((nn + 1) * 8);
  w.blocksum = (uint64_t*)take(((nn + kScanTile - 1) / kScanTile + 1) * 8);
  for (int i = 0; i < 2; ++i) w.tkeys[i] = (uint32_t*)take(mp * 4);
  w.tvals = (uint32_t*)take(mp * 4);
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
    e = hipMemsetAsync(w.offsets, 0, 8, st);
  }
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t bin_emit_and_sort(const ngs_projected& p, int n, const DevCam& cam, int64_t m, const BinWs& w,
                             const ngs_tile_lists& out, hipStream_t st) {
  const int ntiles = cam.tiles_x * cam.tiles_y;
  int bits = 1;
  while ((1 << bits) < ntiles) ++bits;
  const int passes = (bits + 7) / 8;
  const uint32_t* order = w.dvals[1];
  // Choose where emission writes so that the last pass lands in out.gids.
  uint32_t *ek, *ev, *ak, *av, *bk, *bv;
  if (passes % 2 == 1) {
    ek = w.tkeys[1]; ev = w.tvals;
    ak = w.tkeys[0]; av = out.gids;
    bk = w.tkeys[1]; bv = w.tvals;
  } else {
    ek = w.tkeys[1]; ev = out.gids;
    ak = w.tkeys[0]; av = w.tvals;
    bk = w.tkeys[1]; bv = out.gids;
  }
  hipError_t e = hipMemsetAsync(out.ranges, 0, sizeof(uint32_t) * 2 * (size_t)ntiles, st);
  if (e != hipSuccess) return e;
  e = hipMemcpyAsync(out.n_pairs, w.offsets + n, sizeof(int64_t), hipMemcpyDeviceToDevice, st);
  if (e != hipSuccess) return e;
  if (m == 0) return hipSuccess;
  {
    ProfScope ps(kProfEmit, st);
    hipLaunchKernelGGL(k_emit, dim3((n + kEmitRanks - 1) / kEmitRanks), dim3(kEmitRanks), 0, st, n, order, w.offsets, p.rect,
                       cam.tiles_x, ek, ev);
  }
  uint32_t *ko, *vo;
  e = radix_sort_pairs(ek, ev, ak, av, bk, bv, (size_t)m, 0, bits, w.sort, st, &ko, &vo, kProfTileHist);
  if (e != hipSuccess) return e;
  if (vo != out.gids) return hipErrorInvalidValue;
  const unsigned gb = (unsigned)((m + 255) / 256);
  {
    ProfScope ps(kProfRanges, st);
    hipLaunchKernelGGL(k_ranges, dim3(gb), dim3(256), 0, st, ko, m, out.ranges, ntiles);
  }
  if (out.keys) {
    ProfScope ps(kProfKeys64, st);
    hipLaunchKernelGGL(k_keys64, dim3(gb), dim3(256), 0, st, ko, out.gids, p.zkey, m, out.keys);
  }
  return hipGetLastError();
}

}  // namespace ngs
