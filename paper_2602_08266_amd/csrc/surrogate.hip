// surrogate.hip -- learned view scorer: a small convolutional network that predicts a view's
// next-best-view score from low-resolution rendered feature maps (depth, final transmittance,
// argmax object id, mean confidence). Not part of the paper: an addition whose ranking is
// judged by, and falls back to, the exact information gain.
//
// Network (fixed): four 3x3 convolutions with stride 2 and padding 1 (4 -> 32 -> 64 -> 128 ->
// 128 channels, 60x80 -> 30x40 -> 15x20 -> 8x10 -> 4x5), ReLU, global average pool, then
// 128 -> 128 (ReLU) -> 1. Activations are channel-major [C][B][H][W]. Every convolution and
// fully connected layer is a GEMM on BF16 operands with FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x32_bf16): forward Z = W * col(X); backward dW = dZ * col(X)^T and
// col(dX) = W^T * dZ. The BF16 rounding points are the GEMM operands: weights, the im2col of
// activations, the pooled and hidden activations, and the pre-activation gradients.
#include <hip/hip_runtime.h>

#include <cmath>

#include "common.hpp"

namespace ngs {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  const uint32_t u = __float_as_uint(f);
  return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// ---- GEMM: C[M][N] = op(A)[M][K] * op(B)[K][N] + beta * C, BF16 in, FP32 out ----------
// op(A) = A (row-major, lda) or A^T (A stored [K][M]); op(B) = B ([K][N]) or B^T ([N][K]).
// 64 x 64 block tile, K step 32, four wavefronts each owning a 32 x 32 quarter as 2 x 2
// MFMA tiles of 16 x 16. For v_mfma_f32_16x16x32_bf16 lane l supplies row (l mod 16) of A
// and column (l mod 16) of B at k = 8 (l / 16) ... +7, and receives C rows 4 (l / 16) ... +3
// of column (l mod 16). Long-K products with few output tiles (the weight gradients, whose K
// is batch x pixels) split K over grid.z: each split writes its partial tile to a workspace
// slab and a second kernel sums the slabs in split order, so results do not depend on timing.
constexpr int kGM = 64, kGN = 64, kGK = 32, kGPad = 8;
constexpr int kMaxSplits = 64;

// Eight consecutive BF16 words of a row (row-major source with leading dimension ld): one
// 16-byte load when all eight lie in bounds and the address is 16-byte aligned, else word by
// word (zero past the bounds).
__device__ __forceinline__ uint4 load8(const uint16_t* __restrict__ src, int row, int rows, int col, int cols,
                                       int ld) {
  uint4 v = make_uint4(0u, 0u, 0u, 0u);
  if (row >= rows || col >= cols) return v;
  const uint16_t* p = src + (size_t)row * ld + col;
  if (col + 8 <= cols && (reinterpret_cast<uintptr_t>(p) & 15u) == 0u) return *reinterpret_cast<const uint4*>(p);
  uint16_t w[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) w[i] = col + i < cols ? p[i] : (uint16_t)0;
  v.x = w[0] | ((uint32_t)w[1] << 16); v.y = w[2] | ((uint32_t)w[3] << 16);
  v.z = w[4] | ((uint32_t)w[5] << 16); v.w = w[6] | ((uint32_t)w[7] << 16);
  return v;
}

// Stages one operand tile (64 rows of the output dimension x 32 of K) from global memory: each
// of the 256 threads loads eight consecutive words of the source's contiguous dimension. With
// K contiguous (T = false for A, true for B) they are eight k of one row and go to LDS as one
// 16-byte store; with the output dimension contiguous they are eight rows at one k and go to
// LDS word by word (the tile is [row][k] either way, as the MFMA operands read it).
template <bool KCONTIG>
__device__ __forceinline__ uint4 stage_load(const uint16_t* __restrict__ src, int ld, int r0, int rows, int k0,
                                            int kend, int tid) {
  if (KCONTIG) {
    const int rr = tid >> 2, kk = (tid & 3) * 8;
    return load8(src, r0 + rr, rows, k0 + kk, kend, ld);
  }
  const int kk = tid >> 3, rr = (tid & 7) * 8;
  return load8(src, k0 + kk, kend, r0 + rr, rows, ld);
}

template <bool KCONTIG>
__device__ __forceinline__ void stage_store(uint16_t (*dst)[kGK + kGPad], uint4 v, int tid) {
  if (KCONTIG) {
    *reinterpret_cast<uint4*>(&dst[tid >> 2][(tid & 3) * 8]) = v;
  } else {
    const int kk = tid >> 3, rr = (tid & 7) * 8;
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dst[rr + 2 * i][kk] = (uint16_t)(w[i] & 0xFFFFu);
      dst[rr + 2 * i + 1][kk] = (uint16_t)(w[i] >> 16);
    }
  }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const uint16_t* __restrict__ A, int lda,
                                                   const uint16_t* __restrict__ B, int ldb, float* __restrict__ C,
                                                   int ldc, float beta, int kchunk, float* __restrict__ part) {
  __shared__ __align__(16) uint16_t As[kGM][kGK + kGPad];
  __shared__ __align__(16) uint16_t Bs[kGN][kGK + kGPad];
  const int m0 = blockIdx.y * kGM, n0 = blockIdx.x * kGN;
  const int kbeg = blockIdx.z * kchunk, kend = min(K, kbeg + kchunk);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  f32x4 acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // A is [M][K] (K contiguous) unless transposed; B is [K][N] (N contiguous) unless transposed.
  // The next K step's operands are loaded into registers while the current one is multiplied.
  uint4 ra = stage_load<!TA>(A, lda, m0, M, kbeg, kend, tid);
  uint4 rb = stage_load<TB>(B, ldb, n0, N, kbeg, kend, tid);
  for (int k0 = kbeg; k0 < kend; k0 += kGK) {
    stage_store<!TA>(As, ra, tid);
    stage_store<TB>(Bs, rb, tid);
    __syncthreads();
    if (k0 + kGK < kend) {
      ra = stage_load<!TA>(A, lda, m0, M, k0 + kGK, kend, tid);
      rb = stage_load<TB>(B, ldb, n0, N, k0 + kGK, kend, tid);
    }
    const int kb = 8 * (lane >> 4);
#pragma unroll
    for (int mi = 0; mi < 2; ++mi) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + mi * 16 + (lane & 15)][kb]);
#pragma unroll
      for (int ni = 0; ni < 2; ++ni) {
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + ni * 16 + (lane & 15)][kb]);
        acc[mi][ni] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[mi][ni], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int mi = 0; mi < 2; ++mi)
#pragma unroll
    for (int ni = 0; ni < 2; ++ni)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = m0 + wm * 32 + mi * 16 + 4 * (lane >> 4) + i;
        const int col = n0 + wn * 32 + ni * 16 + (lane & 15);
        if (row < M && col < N) {
          if (part) {
            part[((size_t)blockIdx.z * M + row) * N + col] = acc[mi][ni][i];
          } else {
            float* c = C + (size_t)row * ldc + col;
            *c = acc[mi][ni][i] + (beta != 0.f ? beta * *c : 0.f);
          }
        }
      }
}

__global__ void k_splitk_reduce(const float* __restrict__ part, int splits, int M, int N, float* __restrict__ C,
                                int ldc, float beta) {
  const size_t MN = (size_t)M * N;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < MN; i += (size_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < splits; ++z) s += part[(size_t)z * MN + i];
    float* c = C + (i / N) * (size_t)ldc + (i % N);
    *c = s + (beta != 0.f ? beta * *c : 0.f);
  }
}

// Splits of K for an M x N x K product: enough workgroups to cover the chip twice, each split
// at least 8 K steps long.
int splitk_for(int M, int N, int K) {
  const int tiles = ((M + kGM - 1) / kGM) * ((N + kGN - 1) / kGN);
  if (tiles >= 512) return 1;
  int s = std::min(kMaxSplits, (512 + tiles - 1) / tiles);
  s = std::min(s, std::max(1, K / (8 * kGK)));
  return std::max(s, 1);
}

// part: workspace for split-K partials (splitk_for(M, N, K) * M * N floats), or NULL for a
// single pass.
hipError_t gemm(bool ta, bool tb, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                float* C, int ldc, float beta, hipStream_t st, float* part = nullptr) {
  if (M <= 0 || N <= 0) return hipSuccess;
  ProfScope ps(kProfSurGemm, st);
  const int splits = part ? splitk_for(M, N, K) : 1;
  const int kchunk = splits > 1 ? ((K + splits - 1) / splits + kGK - 1) / kGK * kGK : std::max(K, 1);
  const int used = splits > 1 ? (K + kchunk - 1) / kchunk : 1;
  float* pp = used > 1 ? part : nullptr;
  const dim3 grid((N + kGN - 1) / kGN, (M + kGM - 1) / kGM, used);
  if (!ta && !tb) hipLaunchKernelGGL((k_gemm_bf16<false, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, beta, kchunk, pp);
  else if (!ta && tb) hipLaunchKernelGGL((k_gemm_bf16<false, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, beta, kchunk, pp);
  else if (ta && !tb) hipLaunchKernelGGL((k_gemm_bf16<true, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, beta, kchunk, pp);
  else hipLaunchKernelGGL((k_gemm_bf16<true, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, C, ldc, beta, kchunk, pp);
  if (pp) {
    const size_t mn = (size_t)M * N;
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)std::min<size_t>((mn + 255) / 256, 4096)), dim3(256), 0, st,
                       pp, used, M, N, C, ldc, beta);
  }
  return hipGetLastError();
}

// ---- elementwise kernels --------------------------------------------------------------------
constexpr int kEw = 256;
inline dim3 ew_grid(size_t n) { return dim3((unsigned)std::min<size_t>((n + kEw - 1) / kEw, 65536)); }

__global__ void k_to_bf16(const float* __restrict__ x, uint16_t* __restrict__ y, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    y[i] = to_bf16(x[i]);
}

// col[(c * 9 + kh * 3 + kw)][(b * Ho + ho) * Wo + wo] = x[c][b][ho s - 1 + kh][wo s - 1 + kw] (0 outside)
__global__ void k_im2col(const float* __restrict__ x, int C, int B, int H, int W, int s, int Ho, int Wo,
                         uint16_t* __restrict__ col) {
  const size_t N = (size_t)B * Ho * Wo, total = (size_t)C * 9 * N;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int row = (int)(i / N);
    const size_t nn = i % N;
    const int c = row / 9, kh = (row % 9) / 3, kw = row % 3;
    const int b = (int)(nn / ((size_t)Ho * Wo));
    const int r = (int)(nn % ((size_t)Ho * Wo));
    const int h = (r / Wo) * s - 1 + kh, w = (r % Wo) * s - 1 + kw;
    float v = 0.f;
    if (h >= 0 && h < H && w >= 0 && w < W) v = x[(((size_t)c * B + b) * H + h) * W + w];
    col[i] = to_bf16(v);
  }
}

// dx[c][b][h][w] = sum over the (kh, kw, ho, wo) that read x[c][b][h][w] of dcol
__global__ void k_col2im(const float* __restrict__ dcol, int C, int B, int H, int W, int s, int Ho, int Wo,
                         float* __restrict__ dx) {
  const size_t N = (size_t)B * Ho * Wo, total = (size_t)C * B * H * W;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int w = (int)(i % W), h = (int)((i / W) % H);
    const int b = (int)((i / ((size_t)W * H)) % B), c = (int)(i / ((size_t)W * H * B));
    float v = 0.f;
    for (int kh = 0; kh < 3; ++kh) {
      const int hh = h + 1 - kh;
      if (hh < 0 || hh % s) continue;
      const int ho = hh / s;
      if (ho >= Ho) continue;
      for (int kw = 0; kw < 3; ++kw) {
        const int ww = w + 1 - kw;
        if (ww < 0 || ww % s) continue;
        const int wo = ww / s;
        if (wo >= Wo) continue;
        v += dcol[(size_t)(c * 9 + kh * 3 + kw) * N + ((size_t)b * Ho + ho) * Wo + wo];
      }
    }
    dx[i] = v;
  }
}

// y[r][j] += bias[r]; optional ReLU; optional BF16 copy
__global__ void k_bias_act(float* __restrict__ y, const float* __restrict__ bias, int rows, size_t cols, int relu,
                           uint16_t* __restrict__ yb) {
  const size_t total = (size_t)rows * cols;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    float v = y[i] + bias[i / cols];
    if (relu) v = fmaxf(v, 0.f);
    y[i] = v;
    if (yb) yb[i] = to_bf16(v);
  }
}

// dz = dy * (y > 0) (BF16 copy for the GEMMs), db[r] = sum_j dz[r][j]; one block per row
__global__ __launch_bounds__(256) void k_act_bwd(const float* __restrict__ dy, const float* __restrict__ y,
                                                 size_t cols, int relu, uint16_t* __restrict__ dzb,
                                                 float* __restrict__ db) {
  __shared__ float red[256];
  const int r = blockIdx.x;
  float acc = 0.f;
  for (size_t j = threadIdx.x; j < cols; j += 256) {
    const size_t i = (size_t)r * cols + j;
    const float v = (!relu || y[i] > 0.f) ? dy[i] : 0.f;
    dzb[i] = to_bf16(v);
    acc += v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[r] = red[0];
}

// p[c][b] = mean over s of x[c][b][s] (FP32 and BF16)
__global__ void k_pool_fwd(const float* __restrict__ x, int C, int B, int S, float* __restrict__ p,
                           uint16_t* __restrict__ pb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= C * B) return;
  float v = 0.f;
  for (int s = 0; s < S; ++s) v += x[(size_t)i * S + s];
  v /= (float)S;
  p[i] = v;
  pb[i] = to_bf16(v);
}

__global__ void k_pool_bwd(const float* __restrict__ dp, int C, int B, int S, float* __restrict__ dx) {
  const size_t total = (size_t)C * B * S;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x)
    dx[i] = dp[i / S] / (float)S;
}

// loss = mean (pred - t)^2, dpred = 2 (pred - t) / B (single block)
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ pred, const float* __restrict__ t, int B,
                                             float* __restrict__ dpred, float* __restrict__ loss) {
  __shared__ float red[256];
  float acc = 0.f;
  for (int i = threadIdx.x; i < B; i += 256) {
    const float d = pred[i] - t[i];
    dpred[i] = 2.f * d / (float)B;
    acc += d * d;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss) *loss = red[0] / (float)B;
}

// Adam with bias correction; refreshes the BF16 copy of the weight
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       size_t n, float lr, float b1, float b2, float eps, float c1, float c2,
                       uint16_t* __restrict__ wb) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    w[i] = wi;
    if (wb) wb[i] = to_bf16(wi);
  }
}

// Input channels of view `index` from its 80x60-class render: depth / depth_scale,
// final transmittance, argmax object id / k, mean confidence.
__global__ void k_features(const float* __restrict__ depth, const float* __restrict__ tfin,
                           const int32_t* __restrict__ id, const float* __restrict__ kbar, int HW, int B, int index0,
                           float inv_depth, float inv_k, size_t set_stride, float* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= HW) return;
  // view index0 + blockIdx.y reads the image set blockIdx.y * set_stride bytes past the first
  const size_t so = (size_t)blockIdx.y * set_stride;
  depth = (const float*)((const char*)depth + so);
  tfin = (const float*)((const char*)tfin + so);
  id = (const int32_t*)((const char*)id + so);
  kbar = (const float*)((const char*)kbar + so);
  const int index = index0 + (int)blockIdx.y;
  x[((size_t)0 * B + index) * HW + i] = depth[i] * inv_depth;
  x[((size_t)1 * B + index) * HW + i] = tfin[i];
  x[((size_t)2 * B + index) * HW + i] = (float)id[i] * inv_k;
  x[((size_t)3 * B + index) * HW + i] = kbar[i];
}

// Novelty of every Gaussian against the training information: for each output f with block
// dimension d_f, the geometric mean eigenvalue of H_T,g,f relative to the prior lambda,
// exp((logdet H_T,g,f - d_f ln lambda) / d_f), is 1 for a Gaussian no training view touched
// and grows with what the views observed; its reciprocal, averaged over the three outputs and
// scaled by the confidence c_g, is the weight the feature render averages along each ray.
__global__ void k_novelty(int n, int k, const float* __restrict__ conf, const int32_t* __restrict__ slot_of,
                          const double* __restrict__ logdet, int capacity, double ln_lambda, float* __restrict__ out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const int s = slot_of ? slot_of[g] : -1;
  double nu = 1.0;
  if (s >= 0 && s < capacity) {
    const double d[3] = {14.0, 11.0, 11.0 + (double)k};
    nu = 0.0;
    for (int f = 0; f < 3; ++f) nu += exp(-(logdet[(size_t)f * capacity + s] - d[f] * ln_lambda) / d[f]);
    nu *= 1.0 / 3.0;
  }
  out[g] = (float)((double)conf[g] * nu);
}

// ---- network shape and workspace ------------------------------------------------------------
struct ConvShape { int ci, co, h, w, ho, wo; };
constexpr ConvShape kConv[4] = {{4, 32, 60, 80, 30, 40}, {32, 64, 30, 40, 15, 20}, {64, 128, 15, 20, 8, 10},
                                {128, 128, 8, 10, 4, 5}};
constexpr int kWidth = NGS_SUR_WIDTH;

struct SurWs {
  uint16_t* col[4];  // im2col of each conv input [ci * 9][B ho wo]
  float* act[4];     // post-ReLU conv outputs [co][B ho wo]
  float* pool;       // [128][B]
  uint16_t* poolb;
  float* hid;        // [128][B]
  uint16_t* hidb;
  float* pred;       // [B] (fc2 output before the caller's copy)
  float* dz;         // FP32 gradient scratch, the largest activation
  uint16_t* dzb;     // its BF16 copy
  float* dcol;       // [ci * 9][B ho wo] of the largest layer
  float* dact;       // gradient of the current layer input
  uint16_t* xb;      // unused (kept aligned)
  float* part;       // split-K partials of the weight-gradient products
};

// Largest split-K slab set of a weight-gradient product (co x ci*9 per layer, 128 x 128, 1 x 128).
size_t part_floats() {
  size_t m = (size_t)kWidth * kWidth;
  for (int l = 0; l < 4; ++l) m = std::max(m, (size_t)kConv[l].co * kConv[l].ci * 9);
  return (size_t)kMaxSplits * m;
}

size_t al(size_t x) { return (x + 255) / 256 * 256; }

size_t sur_ws_bytes(int B) {
  size_t s = 0;
  size_t max_act = 0, max_col = 0;
  for (int l = 0; l < 4; ++l) {
    const size_t n = (size_t)B * kConv[l].ho * kConv[l].wo;
    s += al((size_t)kConv[l].ci * 9 * n * 2) + al((size_t)kConv[l].co * n * 4);
    max_act = std::max(max_act, (size_t)kConv[l].co * n);
    max_act = std::max(max_act, (size_t)kConv[l].ci * B * kConv[l].h * kConv[l].w);
    max_col = std::max(max_col, (size_t)kConv[l].ci * 9 * n);
  }
  s += 2 * (al((size_t)kWidth * B * 4) + al((size_t)kWidth * B * 2)) + al((size_t)B * 4);
  s += al(max_act * 4) + al(max_act * 2) + al(max_col * 4) + al(max_act * 4);
  s += al(part_floats() * 4);
  return s;
}

SurWs sur_ws_carve(void* ws, int B) {
  char* p = static_cast<char*>(ws);
  auto take = [&](size_t b) { char* r = p; p += al(b); return r; };
  SurWs w;
  size_t max_act = 0, max_col = 0;
  for (int l = 0; l < 4; ++l) {
    const size_t n = (size_t)B * kConv[l].ho * kConv[l].wo;
    w.col[l] = (uint16_t*)take((size_t)kConv[l].ci * 9 * n * 2);
    w.act[l] = (float*)take((size_t)kConv[l].co * n * 4);
    max_act = std::max(max_act, (size_t)kConv[l].co * n);
    max_act = std::max(max_act, (size_t)kConv[l].ci * B * kConv[l].h * kConv[l].w);
    max_col = std::max(max_col, (size_t)kConv[l].ci * 9 * n);
  }
  w.pool = (float*)take((size_t)kWidth * B * 4);
  w.poolb = (uint16_t*)take((size_t)kWidth * B * 2);
  w.hid = (float*)take((size_t)kWidth * B * 4);
  w.hidb = (uint16_t*)take((size_t)kWidth * B * 2);
  w.pred = (float*)take((size_t)B * 4);
  w.dz = (float*)take(max_act * 4);
  w.dzb = (uint16_t*)take(max_act * 2);
  w.dcol = (float*)take(max_col * 4);
  w.dact = (float*)take(max_act * 4);
  w.xb = nullptr;
  w.part = (float*)take(part_floats() * 4);
  return w;
}

// weight elements of layer l (conv 0..3, fc 4..5) and its output width
inline size_t layer_w(int l) {
  if (l < 4) return (size_t)kConv[l].co * kConv[l].ci * 9;
  return l == 4 ? (size_t)kWidth * kWidth : (size_t)kWidth;
}
inline int layer_out(int l) { return l < 4 ? kConv[l].co : (l == 4 ? kWidth : 1); }

#define SUR_TRY(expr)                      \
  do {                                     \
    hipError_t e_ = (expr);                \
    if (e_ != hipSuccess) return e_;       \
  } while (0)

}  // namespace

hipError_t sur_novelty(const ngs_scene& s, const ngs_hessian* h, float lambda, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_novelty, dim3((s.n + 255) / 256), dim3(256), 0, st, s.n, s.k, s.conf,
                     h ? h->slot_of : nullptr, h ? h->logdet : nullptr, h ? h->capacity : 0,
                     log((double)lambda), out);
  return hipGetLastError();
}

size_t sur_workspace_bytes(int batch) { return sur_ws_bytes(batch); }

hipError_t sur_gemm(bool ta, bool tb, int M, int N, int K, const uint16_t* A, int lda, const uint16_t* B, int ldb,
                    float* C, int ldc, float beta, hipStream_t st) {
  return gemm(ta, tb, M, N, K, A, lda, B, ldb, C, ldc, beta, st);
}

hipError_t sur_sync_bf16(const ngs_sur_params& p, hipStream_t st) {
  for (int l = 0; l < NGS_SUR_LAYERS; ++l) {
    const size_t n = layer_w(l);
    hipLaunchKernelGGL(k_to_bf16, ew_grid(n), dim3(kEw), 0, st, p.w[l], p.w_bf16[l], n);
  }
  return hipGetLastError();
}

hipError_t sur_forward(const ngs_sur_params& p, const float* x, int B, float* pred, void* ws, hipStream_t st) {
  ProfScope ps(kProfSurForward, st);
  SurWs w = sur_ws_carve(ws, B);
  const float* in = x;
  for (int l = 0; l < 4; ++l) {
    const ConvShape& c = kConv[l];
    const size_t n = (size_t)B * c.ho * c.wo;
    hipLaunchKernelGGL(k_im2col, ew_grid((size_t)c.ci * 9 * n), dim3(kEw), 0, st, in, c.ci, B, c.h, c.w, 2, c.ho,
                       c.wo, w.col[l]);
    SUR_TRY(hipGetLastError());
    SUR_TRY(gemm(false, false, c.co, (int)n, c.ci * 9, p.w_bf16[l], c.ci * 9, w.col[l], (int)n, w.act[l], (int)n,
                 0.f, st));
    hipLaunchKernelGGL(k_bias_act, ew_grid((size_t)c.co * n), dim3(kEw), 0, st, w.act[l], p.b[l], c.co, n, 1,
                       (uint16_t*)nullptr);
    in = w.act[l];
  }
  const int S = kConv[3].ho * kConv[3].wo;
  hipLaunchKernelGGL(k_pool_fwd, dim3((kWidth * B + 255) / 256), dim3(256), 0, st, w.act[3], kWidth, B, S, w.pool,
                     w.poolb);
  SUR_TRY(gemm(false, false, kWidth, B, kWidth, p.w_bf16[4], kWidth, w.poolb, B, w.hid, B, 0.f, st));
  hipLaunchKernelGGL(k_bias_act, ew_grid((size_t)kWidth * B), dim3(kEw), 0, st, w.hid, p.b[4], kWidth, (size_t)B, 1,
                     w.hidb);
  SUR_TRY(gemm(false, false, 1, B, kWidth, p.w_bf16[5], kWidth, w.hidb, B, w.pred, B, 0.f, st));
  hipLaunchKernelGGL(k_bias_act, ew_grid((size_t)B), dim3(kEw), 0, st, w.pred, p.b[5], 1, (size_t)B, 0,
                     (uint16_t*)nullptr);
  SUR_TRY(hipMemcpyAsync(pred, w.pred, (size_t)B * 4, hipMemcpyDeviceToDevice, st));
  return hipGetLastError();
}

hipError_t sur_backward(const ngs_sur_params& p, const float* x, int B, const float* dpred, const ngs_sur_params& g,
                        void* ws, hipStream_t st) {
  ProfScope ps(kProfSurBackward, st);
  SurWs w = sur_ws_carve(ws, B);
  // fc2: dz = dpred (no activation)
  hipLaunchKernelGGL(k_act_bwd, dim3(1), dim3(256), 0, st, dpred, w.pred, (size_t)B, 0, w.dzb, g.b[5]);
  SUR_TRY(gemm(false, true, 1, kWidth, B, w.dzb, B, w.hidb, B, g.w[5], kWidth, 0.f, st, w.part));          // dW = dz hid^T
  SUR_TRY(gemm(true, false, kWidth, B, 1, p.w_bf16[5], kWidth, w.dzb, B, w.dact, B, 0.f, st));      // dhid = W^T dz
  // fc1
  hipLaunchKernelGGL(k_act_bwd, dim3(kWidth), dim3(256), 0, st, w.dact, w.hid, (size_t)B, 1, w.dzb, g.b[4]);
  SUR_TRY(gemm(false, true, kWidth, kWidth, B, w.dzb, B, w.poolb, B, g.w[4], kWidth, 0.f, st, w.part));
  SUR_TRY(gemm(true, false, kWidth, B, kWidth, p.w_bf16[4], kWidth, w.dzb, B, w.dz, B, 0.f, st));   // dpool
  const int S = kConv[3].ho * kConv[3].wo;
  hipLaunchKernelGGL(k_pool_bwd, ew_grid((size_t)kWidth * B * S), dim3(kEw), 0, st, w.dz, kWidth, B, S, w.dact);
  for (int l = 3; l >= 0; --l) {
    const ConvShape& c = kConv[l];
    const size_t n = (size_t)B * c.ho * c.wo;
    hipLaunchKernelGGL(k_act_bwd, dim3(c.co), dim3(256), 0, st, w.dact, w.act[l], n, 1, w.dzb, g.b[l]);
    SUR_TRY(hipGetLastError());
    SUR_TRY(gemm(false, true, c.co, c.ci * 9, (int)n, w.dzb, (int)n, w.col[l], (int)n, g.w[l], c.ci * 9, 0.f, st,
                 w.part));
    if (l == 0) break;
    SUR_TRY(gemm(true, false, c.ci * 9, (int)n, c.co, p.w_bf16[l], c.ci * 9, w.dzb, (int)n, w.dcol, (int)n, 0.f, st));
    hipLaunchKernelGGL(k_col2im, ew_grid((size_t)c.ci * B * c.h * c.w), dim3(kEw), 0, st, w.dcol, c.ci, B, c.h, c.w,
                       2, c.ho, c.wo, w.dact);
  }
  (void)x;
  return hipGetLastError();
}

hipError_t sur_mse(const float* pred, const float* target, int B, float* dpred, float* loss, hipStream_t st) {
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, st, pred, target, B, dpred, loss);
  return hipGetLastError();
}

hipError_t sur_adam(const ngs_sur_params& p, const ngs_sur_params& g, const ngs_sur_params& m,
                    const ngs_sur_params& v, float lr, float b1, float b2, float eps, int step, hipStream_t st) {
  const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
  for (int l = 0; l < NGS_SUR_LAYERS; ++l) {
    const size_t nw = layer_w(l), nb = (size_t)layer_out(l);
    hipLaunchKernelGGL(k_adam, ew_grid(nw), dim3(kEw), 0, st, p.w[l], g.w[l], m.w[l], v.w[l], nw, lr, b1, b2, eps, c1,
                       c2, p.w_bf16[l]);
    hipLaunchKernelGGL(k_adam, ew_grid(nb), dim3(kEw), 0, st, p.b[l], g.b[l], m.b[l], v.b[l], nb, lr, b1, b2, eps, c1,
                       c2, (uint16_t*)nullptr);
  }
  return hipGetLastError();
}

hipError_t sur_features(const ngs_image& img, int W, int H, int k, float depth_scale, float* x, int B, int index,
                        int views, size_t set_stride, hipStream_t st) {
  const int HW = W * H;
  if (views < 1) return hipSuccess;
  hipLaunchKernelGGL(k_features, dim3((HW + 255) / 256, views), dim3(256), 0, st, img.depth, img.t_final,
                     img.argmax_id, img.mean_conf, HW, B, index, 1.f / depth_scale, 1.f / (float)k, set_stride, x);
  return hipGetLastError();
}

}  // namespace ngs
