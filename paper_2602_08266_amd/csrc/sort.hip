// sort.hip -- stable LSD radix sort of (u32 key, u32 value) pairs, 8-bit digits.
//
// One pass = histogram (per block digit counts), per-digit scan across blocks, scatter.
// The scatter ranks keys inside each wavefront with ballot match masks (8 ballots give the
// set of lanes sharing a digit), so equal digits keep their input order across lanes,
// waves, rounds and blocks: the pass is stable, and successive passes from the least
// significant digit sort by the whole key with ties kept in input order.
#include "common.hpp"

namespace ngs {
namespace {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTileElems = kSortThreads * kSortItems;  // 2048 keys per block
constexpr int kWavesPerBlock = kSortThreads / kWave;

// Every kernel below sorts grid.y arrays at once: view v's arrays lie v * vs bytes past those
// passed.
__global__ __launch_bounds__(kSortThreads) void k_hist(const uint32_t* keys_, size_t n, int shift, uint32_t* hist_,
                                                       size_t nblocks, size_t vs) {
  const uint32_t* __restrict__ keys = vp(keys_, vs);
  uint32_t* __restrict__ hist = vp(hist_, vs);
  __shared__ uint32_t h[kRadix];
  h[threadIdx.x] = 0;
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * kSortTileElems;
  if (shift < 24) {
#pragma unroll 4
    for (int j = 0; j < kSortItems; ++j) {
      const size_t i = base + (size_t)j * kSortThreads + threadIdx.x;
      if (i < n) atomicAdd(&h[(keys[i] >> shift) & (kRadix - 1)], 1u);
    }
  } else {
    // the top digit of depth keys takes a handful of values: lanes with equal digits are
    // grouped by ballots and one of them adds the group's count (no same-address LDS atomics)
    const int lane = threadIdx.x % kWave;
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    for (int j = 0; j < kSortItems; ++j) {
      const size_t i = base + (size_t)j * kSortThreads + threadIdx.x;
      const bool valid = i < n;
      const uint32_t d = valid ? (keys[i] >> shift) & (kRadix - 1) : 0u;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < kRadixBits; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
      }
      if (valid && (peers & lt_mask) == 0ull) atomicAdd(&h[d], (uint32_t)__popcll(peers));
    }
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Inclusive sum over the wavefront's lanes 0..l, by DPP moves: a scan within each row of 16
// lanes (shifts 1, 2, 4, 8), then the row totals carried into the later rows (row_bcast 15
// and 31).
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, false);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return x;
}

// Block-wide exclusive scan of one value per thread (256 threads); returns the total. Each
// wavefront scans its 64 values, then the earlier wavefronts' totals are added.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* sm, uint32_t* total) {
  const int t = threadIdx.x, wave = t / kWave;
  const uint32_t incl = wave_inclusive_scan(v);
  if (t % kWave == kWave - 1) sm[wave] = incl;
  __syncthreads();
  uint32_t before = 0u, all = 0u;
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) {
    const uint32_t s = sm[w];
    before += w < wave ? s : 0u;
    all += s;
  }
  *total = all;
  __syncthreads();  // sm is reused by the next scan
  return before + incl - v;
}

// One block per digit: exclusive scan of that digit's counts across blocks, in place;
// rowtot[d] = total count of digit d.
__global__ __launch_bounds__(kSortThreads) void k_scan_rows(uint32_t* hist_, size_t nblocks, uint32_t* rowtot_,
                                                            size_t vs) {
  uint32_t* __restrict__ hist = vp(hist_, vs);
  uint32_t* __restrict__ rowtot = vp(rowtot_, vs);
  __shared__ uint32_t sm[kSortThreads];
  uint32_t* row = hist + (size_t)blockIdx.x * nblocks;
  uint32_t carry = 0;
  for (size_t b0 = 0; b0 < nblocks; b0 += kSortThreads) {
    const size_t i = b0 + threadIdx.x;
    const uint32_t v = (i < nblocks) ? row[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan(v, sm, &tot);
    if (i < nblocks) row[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) rowtot[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kSortThreads) void k_scatter(const uint32_t* kin_, const uint32_t* vin_, size_t n,
                                                          int shift, const uint32_t* hist_, size_t nblocks,
                                                          const uint32_t* rowtot_, uint32_t* kout_, uint32_t* vout_,
                                                          const uint2* rin_, uint2* rout_, size_t vs) {
  const uint32_t* __restrict__ kin = vp(kin_, vs);
  const uint32_t* __restrict__ vin = vp(vin_, vs);
  const uint32_t* __restrict__ hist = vp(hist_, vs);
  const uint32_t* __restrict__ rowtot = vp(rowtot_, vs);
  uint32_t* __restrict__ kout = vp(kout_, vs);
  uint32_t* __restrict__ vout = vp(vout_, vs);
  const uint2* __restrict__ rin = vp(rin_, vs);
  uint2* __restrict__ rout = vp(rout_, vs);
  // The block's 2048 pairs are first ranked into digit order in LDS (stable), then streamed
  // out: consecutive lanes write consecutive positions of each digit's run. Wavefront w owns
  // the block's pairs [512 w, 512 w + 512), item j of lane l being pair 512 w + 64 j + l, so
  // (wavefront, item, lane) is the input order: each wavefront ranks its items in turn against
  // its own running digit counts (no workgroup barrier per item), and one scan over
  // (digit, wavefront) then places the wavefronts' runs one after another.
  constexpr int kWaveElems = kSortTileElems / kWavesPerBlock;
  __shared__ uint32_t sm[kSortThreads];
  __shared__ uint32_t gbase[kRadix];           // global position of this block's first key of digit d
  __shared__ uint32_t lstart[kRadix];          // local position of the first key of digit d
  __shared__ uint32_t wcnt[kWavesPerBlock][kRadix];  // per wavefront: digit counts, then its run start
  __shared__ uint32_t sk[kSortTileElems], sv[kSortTileElems];
  const int t = threadIdx.x;
  const int wave = t / kWave;
  const int lane = t % kWave;
  const size_t blk = (size_t)blockIdx.x * kSortTileElems;
  const int cnt = (int)min((size_t)kSortTileElems, n - blk);
  uint32_t keys[kSortItems], vals[kSortItems], idx[kSortItems];
#pragma unroll
  for (int w = 0; w < kWavesPerBlock; ++w) wcnt[w][t] = 0u;
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int li = wave * kWaveElems + j * kWave + lane;
    keys[j] = li < cnt ? kin[blk + li] : 0u;
    vals[j] = li < cnt ? (vin ? vin[blk + li] : (uint32_t)(blk + li)) : 0u;
  }
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  uint32_t* wc = wcnt[wave];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const bool valid = wave * kWaveElems + j * kWave + lane < cnt;
    const uint32_t d = (keys[j] >> shift) & (kRadix - 1);
    // lanes holding the same digit (8 ballots), this lane's rank among them, the lowest leads
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t before = wc[d];  // read by every lane before the leader advances it
    idx[j] = before + (uint32_t)__popcll(peers & lt_mask);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    if (valid && (peers & lt_mask) == 0ull) wc[d] = before + (uint32_t)__popcll(peers);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  }
  __syncthreads();
  {
    // thread t = digit: the block's count of it, its local start, and each wavefront's run start
    uint32_t tot_d = 0u;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) tot_d += wcnt[w][t];
    uint32_t tot;
    uint32_t run = block_exclusive_scan(tot_d, sm, &tot);
    lstart[t] = run;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) {
      const uint32_t c = wcnt[w][t];
      wcnt[w][t] = run;
      run += c;
    }
    const uint32_t digit_start = block_exclusive_scan(rowtot[t], sm, &tot);
    gbase[t] = digit_start + hist[(size_t)t * nblocks + blockIdx.x];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    if (wave * kWaveElems + j * kWave + lane < cnt) {
      const uint32_t lp = wc[(keys[j] >> shift) & (kRadix - 1)] + idx[j];
      sk[lp] = keys[j];
      sv[lp] = vals[j];
    }
  }
  __syncthreads();
  // every gathered record is loaded before anything is stored (a wait for loads issued after
  // stores would also wait for the stores)
  uint32_t ok[kSortItems], ov[kSortItems];
  uint2 orr[kSortItems];
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int i = t + j * kSortThreads;
    ok[j] = i < cnt ? sk[i] : 0u;
    ov[j] = i < cnt ? sv[i] : 0u;
    if (rout && i < cnt) orr[j] = rin[ov[j]];  // an 8-byte record of the value's, carried into sorted order
  }
#pragma unroll
  for (int j = 0; j < kSortItems; ++j) {
    const int i = t + j * kSortThreads;
    if (i < cnt) {
      const uint32_t d = (ok[j] >> shift) & (kRadix - 1);
      const uint32_t pos = gbase[d] + ((uint32_t)i - lstart[d]);
      kout[pos] = ok[j];
      vout[pos] = ov[j];
      if (rout) rout[pos] = orr[j];
    }
  }
}

__global__ void k_iota(uint32_t* v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (uint32_t)i;
}
__global__ void k_fill_u32(uint32_t* v_, uint32_t x, size_t n, size_t vs) {
  uint32_t* v = vp(v_, vs);
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = x;
}
__global__ void k_fill_i32(int32_t* v, int32_t x, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = x;
}
__global__ void k_copy_u32(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

size_t sort_blocks_for(size_t n) { return (n + kSortTileElems - 1) / kSortTileElems; }

hipError_t launch_iota(uint32_t* v, size_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  ProfScope ps(kProfFill, st);
  hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v, n);
  return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t* v, uint32_t x, size_t n, hipStream_t st, int g, size_t vs) {
  if (!n) return hipSuccess;
  ProfScope ps(kProfFill, st);
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256), g), dim3(256), 0, st, v, x, n, vs);
  return hipGetLastError();
}
hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, size_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  ProfScope ps(kProfFill, st);
  hipLaunchKernelGGL(k_copy_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t* v, int32_t x, size_t n, hipStream_t st) {
  if (!n) return hipSuccess;
  ProfScope ps(kProfFill, st);
  hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, v, x, n);
  return hipGetLastError();
}

// Sorts bits [begin_bit, end_bit) of the keys; the result is in (*keys_out, *vals_out),
// which is one of the two ping-pong buffers (a, b), for g arrays at once (view v's at v * vs
// bytes past those passed). The inputs are only read; vals_in NULL
// stands for the values 0, 1, ..., n - 1 (the keys' own positions). With rec_in (8-byte
// records indexed by value) the last pass also writes rec_sorted[i] = rec_in[value of i].
hipError_t radix_sort_pairs(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_a,
                            uint32_t* vals_a, uint32_t* keys_b, uint32_t* vals_b, size_t n, int begin_bit,
                            int end_bit, const SortWs& ws, hipStream_t st, uint32_t** keys_out,
                            uint32_t** vals_out, int prof_base, const void* rec_in, void* rec_sorted, int g,
                            size_t vs) {
  const size_t nb = sort_blocks_for(n);
  if (nb > ws.max_blocks) return hipErrorInvalidValue;
  const uint32_t* kin = keys_in;
  const uint32_t* vin = vals_in;
  uint32_t* kdst = keys_a;
  uint32_t* vdst = vals_a;
  *keys_out = const_cast<uint32_t*>(keys_in);
  *vals_out = const_cast<uint32_t*>(vals_in);
  if (n == 0) return hipSuccess;
  for (int shift = begin_bit; shift < end_bit; shift += kRadixBits) {
    {
      ProfScope ps(prof_base, st);
      hipLaunchKernelGGL(k_hist, dim3((unsigned)nb, g), dim3(kSortThreads), 0, st, kin, n, shift, ws.hist, nb, vs);
    }
    {
      ProfScope ps(prof_base + 1, st);
      hipLaunchKernelGGL(k_scan_rows, dim3(kRadix, g), dim3(kSortThreads), 0, st, ws.hist, nb, ws.rowtot, vs);
    }
    {
      ProfScope ps(prof_base + 2, st);
      const bool last = shift + kRadixBits >= end_bit;
      hipLaunchKernelGGL(k_scatter, dim3((unsigned)nb, g), dim3(kSortThreads), 0, st, kin, vin, n, shift, ws.hist, nb,
                         ws.rowtot, kdst, vdst, last ? static_cast<const uint2*>(rec_in) : nullptr,
                         last ? static_cast<uint2*>(rec_sorted) : nullptr, vs);
    }
    *keys_out = kdst;
    *vals_out = vdst;
    kin = kdst;
    vin = vdst;
    if (kdst == keys_a) { kdst = keys_b; vdst = vals_b; } else { kdst = keys_a; vdst = vals_a; }
  }
  return hipGetLastError();
}

}  // namespace ngs
