// project.hip -- per-scene precompute (softmax, confidence) and per-view projection.
//
// Compiled with -ffp-contract=off: the FP64 key path below (depth, 2D mean, EWA covariance,
// radius, tile rect) is evaluated operation by operation in a fixed order, so that the
// depth keys and tile rects it produces are reproducible bit for bit by any IEEE-754 FP64
// evaluation of the same sequence.
#include "common.hpp"

namespace ngs {
namespace {

// Sigma3 = Rg diag(s^2) Rg^T of Gaussian g in FP64, in a fixed order: s = exp(log-scale),
// the quaternion normalised by its norm, Rg from it, then each entry summed over k in order.
__device__ inline void cov3_of(int n, int g, const float* __restrict__ log_scale, const float* __restrict__ rot,
                               double S3[9]) {
  const double s0 = exp((double)log_scale[g]), s1 = exp((double)log_scale[n + g]),
               s2 = exp((double)log_scale[2 * n + g]);
  const double sc2[3] = {s0 * s0, s1 * s1, s2 * s2};
  const double qw = rot[g], qx = rot[n + g], qy = rot[2 * n + g], qz = rot[3 * n + g];
  const double qn = sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
  const double w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
  double Rg[9];
  Rg[0] = 1.0 - 2.0 * (y * y + z * z); Rg[1] = 2.0 * (x * y - w * z);       Rg[2] = 2.0 * (x * z + w * y);
  Rg[3] = 2.0 * (x * y + w * z);       Rg[4] = 1.0 - 2.0 * (x * x + z * z); Rg[5] = 2.0 * (y * z - w * x);
  Rg[6] = 2.0 * (x * z - w * y);       Rg[7] = 2.0 * (y * z + w * x);       Rg[8] = 1.0 - 2.0 * (x * x + y * y);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc = acc + (Rg[3 * i + k] * sc2[k]) * Rg[3 * j + k];
      S3[3 * i + j] = acc;
    }
}

// p = softmax(o) (Sec. III-A.1), sigma = sigmoid(opacity logit), kappa = max_k p,
// label = argmax_k o (identical to argmax_k p, lowest k on ties), and the confidence
// c_g of Eq. 7 -- or Eq. 12 when a target object is given.
__global__ __launch_bounds__(256) void k_prepare(int n, int k, const float* __restrict__ logit,
                                                 const float* __restrict__ op_logit, float alpha_obj,
                                                 float alpha_opa, int target, float* __restrict__ prob,
                                                 float* __restrict__ opacity, float* __restrict__ kappa,
                                                 float* __restrict__ conf, int32_t* __restrict__ label,
                                                 const float* __restrict__ log_scale, const float* __restrict__ rot,
                                                 double* __restrict__ cov3) {
  // the block's probability rows are staged in LDS (row stride k + 1 against bank conflicts)
  // and written out as one contiguous, coalesced run
  extern __shared__ float pst[];
  const int g0 = blockIdx.x * blockDim.x;
  const int g = g0 + threadIdx.x;
  const int nb = min((int)blockDim.x, n - g0);
  if (g < n) {
    float mx = logit[g];
    int am = 0;
    for (int c = 1; c < k; ++c) {
      const float v = logit[(size_t)c * n + g];
      if (v > mx) { mx = v; am = c; }
    }
    float z = 0.f;
    for (int c = 0; c < k; ++c) z += expf(logit[(size_t)c * n + g] - mx);
    const float inv = 1.f / z;
    for (int c = 0; c < k; ++c) pst[threadIdx.x * (k + 1) + c] = expf(logit[(size_t)c * n + g] - mx) * inv;
    const float sig = 1.f / (1.f + expf(-op_logit[g]));
    const float kap = inv;  // exp(0) / z at the argmax
    opacity[g] = sig;
    kappa[g] = kap;
    label[g] = am;
    float c;
    if (target < 0) {
      c = powf(kap, -alpha_obj) * powf(sig, -alpha_opa);
    } else {
      c = (am == target) ? powf(expf(logit[(size_t)target * n + g] - mx) * inv, -alpha_obj) * powf(sig, -alpha_opa)
                         : 0.f;
    }
    conf[g] = c;
    if (cov3) {
      double S3[9];
      cov3_of(n, g, log_scale, rot, S3);
      for (int i = 0; i < 9; ++i) cov3[(size_t)i * n + g] = S3[i];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nb * k; i += blockDim.x) prob[(size_t)g0 * k + i] = pst[(i / k) * (k + 1) + i % k];
}

// floor(v / tile) clamped to [-1, lim]. The tile size is a power of two (16), so v * (1 / tile)
// is exactly v / tile and the multiply gives the same bits as the division.
__device__ inline int tile_floor(double v, double inv_tile, int lim) {
  double f = floor(v * inv_tile);
  if (f < -1.0) f = -1.0;
  if (f > (double)lim) f = (double)lim;
  return (int)f;
}

// One thread per Gaussian. FP64 key path in the order: X = R mu + t (row by row,
// left to right), Z; m = (f X / Z) + c; Sigma3 (cov3_of, or the scene's copy); T = Jp R; M = T Sigma3;
// Sigma2 = M T^T; +eps on the diagonal; conic; lambda_max; radius; rect.
// Views of a group are the fastest-moving part of the block index (block b: view b % nv,
// Gaussians from 256 (b / nv)), so the views of one range of Gaussians run together and read
// its scene entries from the L2 once.
__global__ __launch_bounds__(256) void k_project(int n, const float* __restrict__ mean,
                                                 const float* __restrict__ log_scale,
                                                 const float* __restrict__ rot, const double* __restrict__ cov3,
                                                 GroupCams gc, int nv, size_t vs,
                                                 double z_near, double eps2d, double inv_tile, float* mean2d_,
                                                 float* conic_, float* depth_, uint32_t* zkey_, int16_t* rect_,
                                                 uint32_t* count_, const float* __restrict__ opacity, float cutoff_q,
                                                 float4* splat_, int tight, const float* __restrict__ conf,
                                                 int32_t* tflag_) {
  const int v = blockIdx.x % nv;
  const int g = (blockIdx.x / nv) * blockDim.x + threadIdx.x;
  if (g >= n) return;
  const DevCam cam = gc.c[v];
  const size_t off = (size_t)v * vs;
  float* __restrict__ mean2d = mean2d_ ? (float*)((char*)mean2d_ + off) : nullptr;
  float* __restrict__ conic = conic_ ? (float*)((char*)conic_ + off) : nullptr;
  float* __restrict__ depth = (float*)((char*)depth_ + off);
  uint32_t* __restrict__ zkey = (uint32_t*)((char*)zkey_ + off);
  int16_t* __restrict__ rect = (int16_t*)((char*)rect_ + off);
  uint32_t* __restrict__ count = (uint32_t*)((char*)count_ + off);
  float4* __restrict__ splat = splat_ ? (float4*)((char*)splat_ + off) : nullptr;
  double R[9];
  for (int i = 0; i < 9; ++i) R[i] = (double)cam.R[i];
  const double mu0 = mean[g], mu1 = mean[n + g], mu2 = mean[2 * n + g];
  double X[3];
  for (int i = 0; i < 3; ++i) X[i] = ((R[3 * i] * mu0 + R[3 * i + 1] * mu1) + R[3 * i + 2] * mu2) + (double)cam.t[i];
  const double Z = X[2];
  bool valid = Z > z_near;
  float mxf = 0.f, myf = 0.f, qa = 0.f, qb = 0.f, qc = 0.f;
  int x0 = 0, y0 = 0, x1 = -1, y1 = -1;
  if (valid) {
    const double fx = cam.fx, fy = cam.fy;
    const double mx = (fx * X[0]) / Z + (double)cam.cx;
    const double my = (fy * X[1]) / Z + (double)cam.cy;
    double S3[9];
    if (cov3) {  // the scene's precomputed Sigma3: the same bits as cov3_of
      for (int i = 0; i < 9; ++i) S3[i] = cov3[(size_t)i * n + g];
    } else {
      cov3_of(n, g, log_scale, rot, S3);
    }
    const double Jp[6] = {fx / Z, 0.0, -(fx * X[0]) / (Z * Z), 0.0, fy / Z, -(fy * X[1]) / (Z * Z)};
    double T[6], M[6];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 3; ++j)
        T[3 * i + j] = ((Jp[3 * i] * R[j] + Jp[3 * i + 1] * R[3 + j]) + Jp[3 * i + 2] * R[6 + j]);
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 3; ++j)
        M[3 * i + j] = ((T[3 * i] * S3[j] + T[3 * i + 1] * S3[3 + j]) + T[3 * i + 2] * S3[6 + j]);
    const double S00 = ((M[0] * T[0] + M[1] * T[1]) + M[2] * T[2]);
    const double S01 = ((M[0] * T[3] + M[1] * T[4]) + M[2] * T[5]);
    const double S11 = ((M[3] * T[3] + M[4] * T[4]) + M[5] * T[5]);
    const double a = S00 + eps2d, b = S01, c = S11 + eps2d;
    const double det = a * c - b * b;
    const double half = (a - c) * 0.5;
    const double lmax = (a + c) * 0.5 + sqrt(half * half + b * b);
    const double r = ceil(3.0 * sqrt(lmax));
    x0 = max(0, tile_floor(mx - r, inv_tile, cam.tiles_x));
    x1 = min(cam.tiles_x - 1, tile_floor(mx + r, inv_tile, cam.tiles_x));
    y0 = max(0, tile_floor(my - r, inv_tile, cam.tiles_y));
    y1 = min(cam.tiles_y - 1, tile_floor(my + r, inv_tile, cam.tiles_y));
    valid = (x0 <= x1) && (y0 <= y1);
    mxf = (float)mx;
    myf = (float)my;
    // the conic only feeds FP32 outputs (not the key path): one reciprocal for its three entries
    const double inv_det = 1.0 / det;
    qa = (float)(c * inv_det);
    qb = (float)(-b * inv_det);
    qc = (float)(a * inv_det);
  }
  // walk record: half-extents of the ellipse q <= cutoff (no entry of a culled Gaussian is walked)
  float hx = -1.f, hy = -1.f;
  if (valid) conic_extent(qa, qb, qc, cutoff_q, &hx, &hy);
  if (tight && valid) {
    // Tile rect of the information walks: only the tiles with a pixel centre inside the
    // ellipse's box (kTile, the only tile size the library accepts). A walk takes an entry for a strip of pixel centres [s0, s1] when
    // mx + hx >= s0 and mx - hx <= s1 in FP32; a tile's centres span [16 t + 0.5, 16 t + 15.5],
    // and those bounds and the FP32 box edges are exact in FP64, so the tiles below are exactly
    // those where the walk can take the entry: the others would be passed over at every pixel.
    // (a degenerate conic has infinite extents: its circle rect is kept)
    if (hx < 1e30f) {
      const double ex0 = (double)(mxf - hx), ex1 = (double)(mxf + hx);
      x0 = max(x0, (int)ceil((ex0 - ((double)kTile - 0.5)) * inv_tile));
      x1 = min(x1, (int)floor((ex1 - 0.5) * inv_tile));
    }
    if (hy < 1e30f) {
      const double ey0 = (double)(myf - hy), ey1 = (double)(myf + hy);
      y0 = max(y0, (int)ceil((ey0 - ((double)kTile - 0.5)) * inv_tile));
      y1 = min(y1, (int)floor((ey1 - 0.5) * inv_tile));
    }
    valid = (x0 <= x1) && (y0 <= y1);
  }
  if (mean2d) {  // the walks of the scoring path read the splat records instead
    mean2d[g] = mxf;
    mean2d[n + g] = myf;
    conic[g] = qa;
    conic[n + g] = qb;
    conic[2 * n + g] = qc;
  }
  const float zf = (float)Z;
  depth[g] = zf;
  zkey[g] = valid ? __float_as_uint(zf) : 0xFFFFFFFFu;
  if (!valid) { x0 = 0; y0 = 0; x1 = -1; y1 = -1; }
  reinterpret_cast<short4*>(rect)[g] = make_short4((short)x0, (short)y0, (short)x1, (short)y1);
  count[g] = valid ? (uint32_t)((x1 - x0 + 1) * (y1 - y0 + 1)) : 0u;
  if (splat) {
    // what a tile walk reads of an entry, in one 32-byte record: 2D mean, conic, opacity and
    // the ellipse's half-extents
    splat[2 * (size_t)g] = make_float4(mxf, myf, qa, qb);
    splat[2 * (size_t)g + 1] = make_float4(qc, valid ? opacity[g] : 0.f, hx, hy);
  }
  if (tflag_) {
    // With a target object: flag the tiles that the rect of a weighted Gaussian (nonzero
    // confidence, reaching a tile) covers, so that the binning and both walks can leave the
    // other tiles at once. The wavefront's live lanes mark one weighted Gaussian's rect at a
    // time (lanes past n have left).
    const uint64_t m0 = __ballot(valid && conf && conf[g] > 0.f);
    if (m0) {
      int32_t* __restrict__ tflag = (int32_t*)((char*)tflag_ + off);
      const int lane = (int)__lane_id();
      const uint64_t act = __ballot(true);
      const int rank = (int)__popcll(act & ((1ull << lane) - 1ull)), na = (int)__popcll(act);
      uint64_t m = m0;
      while (m) {
        const int j = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int X0 = __builtin_amdgcn_readlane(x0, j), Y0 = __builtin_amdgcn_readlane(y0, j);
        const int X1 = __builtin_amdgcn_readlane(x1, j), Y1 = __builtin_amdgcn_readlane(y1, j);
        const int w = X1 - X0 + 1, area = w * (Y1 - Y0 + 1);
        for (int t = rank; t < area; t += na) tflag[(Y0 + t / w) * cam.tiles_x + X0 + t % w] = 1;
      }
    }
  }
}

}  // namespace

hipError_t launch_prepare_scene(const ngs_scene& s, const ngs_ig_params& ig, hipStream_t st) {
  if (s.n == 0) return hipSuccess;
  const int blocks = (s.n + 255) / 256;
  ProfScope ps(kProfPrepare, st);
  hipLaunchKernelGGL(k_prepare, dim3(blocks), dim3(256), (size_t)256 * (s.k + 1) * sizeof(float), st, s.n, s.k,
                     s.obj_logit, s.opacity_logit,
                     ig.alpha_obj, ig.alpha_opa, ig.target_id, s.prob, s.opacity, s.kappa, s.conf, s.label,
                     s.log_scale, s.rot, s.cov3);
  return hipGetLastError();
}

hipError_t launch_project(const ngs_scene& s, const Group& G, const ngs_raster_params& rp,
                          const ngs_projected& out, hipStream_t st, int tight, int32_t* tflag) {
  if (s.n == 0) return hipSuccess;
  const int blocks = (s.n + 255) / 256;
  ProfScope ps(kProfProject, st);
  hipLaunchKernelGGL(k_project, dim3(blocks * G.g), dim3(256), 0, st, s.n, s.mean, s.log_scale, s.rot, s.cov3, G.cams,
                     G.g,
                     G.vs, (double)rp.z_near, (double)rp.eps2d, 1.0 / (double)rp.tile, out.mean2d, out.conic,
                     out.depth, out.zkey, out.rect, out.count, s.opacity, rp.cutoff_q,
                     reinterpret_cast<float4*>(out.splat), tight, s.conf, tflag);
  return hipGetLastError();
}

namespace {
// Sum of the per-Gaussian tile counts (the view's pair count M) into *total.
__global__ __launch_bounds__(256) void k_sum_counts(const uint32_t* __restrict__ count, int n,
                                                    unsigned long long* __restrict__ total) {
  __shared__ unsigned long long sm[256 / 64];
  unsigned long long v = 0ull;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) v += count[i];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  if (threadIdx.x % 64 == 0) sm[threadIdx.x / 64] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long t = sm[0] + sm[1] + sm[2] + sm[3];
    if (t) atomicAdd(total, t);
  }
}
}  // namespace

hipError_t launch_sum_counts(const ngs_projected& p, int n, int64_t* total, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const int blocks = std::min((n + 255) / 256, 1024);
  ProfScope ps(kProfCountScan, st);
  hipLaunchKernelGGL(k_sum_counts, dim3(blocks), dim3(256), 0, st, p.count, n,
                     reinterpret_cast<unsigned long long*>(total));
  return hipGetLastError();
}

}  // namespace ngs
