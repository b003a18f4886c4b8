// finalize.hip -- per touched Gaussian: screen-space statistics -> parameter-space blocks
// (FP64 chain rule), confidence weighting, log-det information gain; training-store updates
// and log-dets; Eq. 10-11 combination and argmax.
//
// Parameter order within a block (Sec. III-B.3 subsets): geometry (mean 3, log-scale 3,
// raw quaternion 4, opacity logit 1), then colour (3) for RGB or object logits (k) for the
// object vector; depth uses geometry only. With u = (m_x, m_y, Q_xx, Q_xy, Q_yy, l) and
// P = du / d theta (6 x 11), the blocks are
//   A_rgb = [[P^T Y_rgb P, P^T X_rgb], [X_rgb^T P, (sum a^2) I_3]]
//   A_d   = P7^T Y_d P7,  P7 = [P; dZ/d theta]
//   A_o   = [[P^T Y_o P, E S], [S E^T, (sum a^2) S S]],   E = P^T X_o,
//   X_o = m1 p^T - Z_o,  S = diag(p) - p p^T (softmax Jacobian).
// Information gain of the view (Eq. 5, 6, 9): sum_g logdet(H_T,g + c_g A_g) - logdet(H_T,g).
//
// The object block is never formed. Its logit part is lambda I + tau S S for every sum of
// such blocks (p is fixed per Gaussian) and its cross part is E S, so the (11 + k)-square
// block is held as (G, E, tau) and its log-det is taken through the Schur complement of
// D = lambda I + tau S S:  logdet D + logdet(G - F^T D^-1 F),  F = S E^T.  S S is diagonal
// plus rank two (diag(p^2) + U C U^T, U = [p, p^2], C = [[p.p, -1], [-1, 0]]), so D^-1 F and
// logdet D follow from the Woodbury identity and the determinant lemma with one 2 x 2
// system: O(11^2 k) work instead of a dense O(k^3) factorisation.
#include "chain.hpp"
#include "common.hpp"

namespace ngs {
namespace {

constexpr int kFinThreads = 128;
constexpr int kSmallL = 16;               // register rows of the dense factorisations (l <= 14)
// Stored object block: G (packed upper 11 x 11), tau, lambda, E (11 x k, row-major), p (k).
constexpr int kObjTau = 66, kObjLam = 67, kObjE = 68;

struct FinShared {
  double A[105];           // packed upper triangle of the RGB (14) or depth (11) block, or G'
  double st[kStatScalar + 6 * NGS_MAX_K];
  double P[7][kNGeo];      // rows 0..5: du/dtheta, row 6: dZ/dtheta
  double Y[7][7];          // current symmetric screen matrix
  double YP[7][kNGeo];
  double G[kNGeo][kNGeo];  // object block: geometry part
  double E[kNGeo][NGS_MAX_K];
  double F[NGS_MAX_K][kNGeo];
  double X[NGS_MAX_K][kNGeo];
  double p[NGS_MAX_K];
  double dinv[NGS_MAX_K];
  double Ep[kNGeo];
  double V[2][kNGeo];
  double W[2][kNGeo];
  double red[4][kFinThreads / kWave];
  double tau;
  double ldD;
  double row[2][kSmallL];  // pivot row of the factorisation (double-buffered)
  int hs;                  // training-store slot
  int hs_new;
};

// Entry (i, j) of the symmetric l x l matrix held as a packed upper triangle.
__device__ __forceinline__ int sym_idx(int i, int j, int l) { return i <= j ? tri_idx(i, j, l) : tri_idx(j, i, l); }

// log det of the symmetric l x l matrix A (packed upper, in LDS) by LDL^T elimination with
// one row per thread held in registers (LM >= l; rows and columns past l act as identity).
// At step j the pivot row j is published in LDS; every later row i subtracts
// (A_ij / A_jj) times it, A_ij being row j's entry i by symmetry of the trailing matrix.
// The pivots' mantissas and exponents are accumulated separately and a single log is taken
// at the end. Returns NaN if a pivot is not positive (matrix not positive definite).
// Called by all kFinThreads threads of the block.
template <int LM>
__device__ double ldl_logdet(const double* A, int l, double (*row)[kSmallL]) {
  const int i = threadIdx.x;
  double a[LM];
#pragma unroll
  for (int c = 0; c < LM; ++c) a[c] = (i < l && c < l) ? A[sym_idx(i, c, l)] : (i == c ? 1.0 : 0.0);
  double mant = 1.0;
  int expo = 0;
  bool bad = false;
  for (int j = 0; j < l; ++j) {
    double* rb = row[j & 1];
    if (i == j) {
#pragma unroll
      for (int c = 0; c < LM; ++c) rb[c] = a[c];
    }
    __syncthreads();
    const double d = rb[j];
    if (!(d > 0.0)) { bad = true; break; }
    int e1, e2;
    const double md = frexp(d, &e1);
    mant = frexp(mant * md, &e2);
    expo += e1 + e2;
    if (i > j && i < l) {
      const double m = rb[i] / d;
#pragma unroll
      for (int c0 = 0; c0 < LM; c0 += 8) {
        if (c0 + 8 > j + 1) {
#pragma unroll
          for (int c = c0; c < c0 + 8 && c < LM; ++c) a[c] -= m * rb[c];
        }
      }
    }
  }
  __syncthreads();
  return bad ? __builtin_nan("") : log(mant) + (double)expo * 0.69314718055994530942;
}

// Upper part of A[0..10][0..10] = Pr^T Y Pr over the first `rows` rows of P (block dim l).
__device__ void geo_block(FinShared& S, int rows, int l) {
  for (int e = threadIdx.x; e < rows * kNGeo; e += kFinThreads) {
    const int a = e / kNGeo, j = e % kNGeo;
    double v = 0.0;
    for (int b = 0; b < rows; ++b) v += S.Y[a][b] * S.P[b][j];
    S.YP[a][j] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < kNGeo * kNGeo; e += kFinThreads) {
    const int i = e / kNGeo, c = e % kNGeo;
    if (c < i) continue;
    double v = 0.0;
    for (int a = 0; a < rows; ++a) v += S.P[a][i] * S.YP[a][c];
    S.A[tri_idx(i, c, l)] = v;
  }
}

__device__ void load_sym(FinShared& S, int base, int dim) {
  if (threadIdx.x == 0) {
    int s = base;
    for (int i = 0; i < dim; ++i)
      for (int j = i; j < dim; ++j) { S.Y[i][j] = S.st[s]; S.Y[j][i] = S.st[s]; ++s; }
  }
  __syncthreads();
}

// Block sums of up to four values per thread; every thread receives the totals.
__device__ void block_sum4(FinShared& S, double (&v)[4]) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double x = v[q];
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off);
    if (lane == 0) S.red[q][wave] = x;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    double x = 0.0;
    for (int w = 0; w < kFinThreads / kWave; ++w) x += S.red[q][w];
    v[q] = x;
  }
  __syncthreads();
}

// log det of the object block held as (G, E, tau) with p = S.p (see the file header).
// G (11 x 11, full) and E (11 x k) are in S; tau > 0.
// trace(A^-1 K) for the packed upper triangle A of an SPD l x l matrix (l <= 14) and K (l x l
// row-major, NULL = identity): Cholesky A = L L^T into work, then per column of K a forward
// and a back substitution; thread 0 computes in FP64, every thread returns the value.
// work holds l * l + 1 doubles.
static_assert(NGS_MAX_K * kNGeo >= 2 * kNGeo * kNGeo + 1 && NGS_MAX_K * kNGeo >= 14 * 14 + 1,
              "S.F doubles as the scratch of trace_inv_prod");
__device__ double trace_inv_prod(const double* A, int l, const double* K, double* work) {
  if (threadIdx.x == 0) {
    double* L = work;
    bool bad = false;
    for (int j = 0; j < l && !bad; ++j) {
      double d = A[tri_idx(j, j, l)];
      for (int q = 0; q < j; ++q) d -= L[j * l + q] * L[j * l + q];
      if (!(d > 0.0)) { bad = true; break; }
      const double ljj = sqrt(d);
      L[j * l + j] = ljj;
      for (int i = j + 1; i < l; ++i) {
        double v = A[tri_idx(j, i, l)];
        for (int q = 0; q < j; ++q) v -= L[i * l + q] * L[j * l + q];
        L[i * l + j] = v / ljj;
      }
    }
    double tr = 0.0;
    if (!bad) {
      double y[kSmallL];
      for (int c = 0; c < l; ++c) {
        for (int i = 0; i < l; ++i) {
          double v = K ? K[i * l + c] : (i == c ? 1.0 : 0.0);
          for (int q = 0; q < i; ++q) v -= L[i * l + q] * y[q];
          y[i] = v / L[i * l + i];
        }
        for (int i = l - 1; i >= 0; --i) {
          double v = y[i];
          for (int q = i + 1; q < l; ++q) v -= L[q * l + i] * y[q];
          y[i] = v / L[i * l + i];
        }
        tr += y[c];
      }
    }
    work[l * l] = bad ? __builtin_nan("") : tr;
  }
  __syncthreads();
  const double r = work[l * l];
  __syncthreads();
  return r;
}

// The object block [[G, E S], [S E^T, D]], D = lambda I + tau S S, reduced to its Schur
// complement: fills S.X = D^-1 F (F = S E^T) and S.A = G - F^T X (packed, 11 x 11), and
// returns logdet D in *ld_d and, when trd is given, trace(D^-1) in *trd (Woodbury).
__device__ void object_schur(FinShared& S, int k, double lambda, double tau, double* ld_d, double* trd) {
  // F = S E^T (k x 11): F[c][r] = p_c (E[r][c] - (E p)_r)
  for (int r = threadIdx.x; r < kNGeo; r += kFinThreads) {
    double v = 0.0;
    for (int c = 0; c < k; ++c) v += S.E[r][c] * S.p[c];
    S.Ep[r] = v;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < k * kNGeo; e += kFinThreads) {
    const int c = e / kNGeo, r = e % kNGeo;
    S.F[c][r] = S.p[c] * (S.E[r][c] - S.Ep[r]);
  }
  // Delta = lambda + tau p^2; Z = U^T Delta^-1 U; sum log Delta; s = p.p
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  double zs[4] = {0.0, 0.0, 0.0, 0.0};
  for (int c = threadIdx.x; c < k; c += kFinThreads) {
    const double pc = S.p[c], p2 = pc * pc;
    const double dl = lambda + tau * p2;
    const double di = 1.0 / dl;
    S.dinv[c] = di;
    acc[0] += p2 * di;            // Z00
    acc[1] += p2 * pc * di;       // Z01
    acc[2] += p2 * p2 * di;       // Z11
    acc[3] += p2;                 // s
    zs[0] += log(dl);
  }
  block_sum4(S, acc);
  block_sum4(S, zs);
  const double z00 = acc[0], z01 = acc[1], z11 = acc[2], sp = acc[3];
  // trace(D^-1) = sum Delta^-1 - trace(W Y), W = B^-1 tau C, Y = U^T Delta^-2 U
  double ty[4] = {0.0, 0.0, 0.0, 0.0};
  if (trd) {
    for (int c = threadIdx.x; c < k; c += kFinThreads) {
      const double pc = S.p[c], p2 = pc * pc, di = S.dinv[c], di2 = di * di;
      ty[0] += di;
      ty[1] += p2 * di2;
      ty[2] += p2 * pc * di2;
      ty[3] += p2 * p2 * di2;
    }
    block_sum4(S, ty);
  }
  // B = I + tau C Z
  const double b00 = 1.0 + tau * (sp * z00 - z01), b01 = tau * (sp * z01 - z11);
  const double b10 = -tau * z00, b11 = 1.0 - tau * z01;
  const double detb = b00 * b11 - b01 * b10;
  *ld_d = zs[0] + log(detb);
  if (trd) {
    const double w00 = tau * (b11 * sp + b01) / detb, w01 = -tau * b11 / detb;
    const double w10 = -tau * (b10 * sp + b00) / detb, w11 = tau * b10 / detb;
    *trd = ty[0] - (w00 * ty[1] + (w01 + w10) * ty[2] + w11 * ty[3]);
  }
  // V = U^T Delta^-1 F (2 x 11); W = B^-1 tau C V; X = Delta^-1 (F - U W)
  for (int e = threadIdx.x; e < 2 * kNGeo; e += kFinThreads) {
    const int q = e / kNGeo, r = e % kNGeo;
    double v = 0.0;
    for (int c = 0; c < k; ++c) {
      const double pc = S.p[c];
      v += (q == 0 ? pc : pc * pc) * S.dinv[c] * S.F[c][r];
    }
    S.V[q][r] = v;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < kNGeo; r += kFinThreads) {
    const double c0 = tau * (sp * S.V[0][r] - S.V[1][r]);  // tau C V
    const double c1 = -tau * S.V[0][r];
    S.W[0][r] = (b11 * c0 - b01 * c1) / detb;
    S.W[1][r] = (-b10 * c0 + b00 * c1) / detb;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < k * kNGeo; e += kFinThreads) {
    const int c = e / kNGeo, r = e % kNGeo;
    const double pc = S.p[c];
    S.X[c][r] = S.dinv[c] * (S.F[c][r] - pc * S.W[0][r] - pc * pc * S.W[1][r]);
  }
  __syncthreads();
  // G' = G - F^T X (upper part, packed, l = 11)
  for (int e = threadIdx.x; e < kNGeo * kNGeo; e += kFinThreads) {
    const int r = e / kNGeo, q = e % kNGeo;
    if (q < r) continue;
    double v = S.G[r][q];
    for (int c = 0; c < k; ++c) v -= S.F[c][r] * S.X[c][q];
    S.A[tri_idx(r, q, kNGeo)] = v;
  }
  __syncthreads();
}

__device__ double object_logdet(FinShared& S, int k, double lambda, double tau) {
  double ld_d;
  object_schur(S, k, lambda, tau, &ld_d, nullptr);
  return ld_d + ldl_logdet<kSmallL>(S.A, kNGeo, S.row);
}

// trace of the object block's inverse from its Schur complement Sigma (in S.A after
// object_schur): trace(M^-1) = trace(D^-1) + trace(Sigma^-1 (I + X^T X)). Uses S.F as scratch.
__device__ double object_trinv_after_schur(FinShared& S, int k, double trd) {
  double* K = &S.F[0][0];
  for (int e = threadIdx.x; e < kNGeo * kNGeo; e += kFinThreads) {
    const int r = e / kNGeo, q = e % kNGeo;
    double v = r == q ? 1.0 : 0.0;
    for (int c = 0; c < k; ++c) v += S.X[c][r] * S.X[c][q];
    K[e] = v;
  }
  __syncthreads();
  return trd + trace_inv_prod(S.A, kNGeo, K, K + kNGeo * kNGeo);
}

__device__ __forceinline__ int block_dim(int f) { return f == 0 ? 14 : kNGeo; }
__device__ __forceinline__ int store_len(int f, int k) { return f == 0 ? 105 : (f == 1 ? 66 : kObjE + 12 * k); }

// The chain-rule matrix P (d(m, Q, l, Z)/d theta, FP64) of every slot with statistics, one
// thread per slot, into the workspace: the straight-line FP64 code would otherwise set the
// register budget of the whole finalize kernel.
__global__ __launch_bounds__(64) void k_fin_chain(int n, const float* __restrict__ mean,
                                                  const float* __restrict__ log_scale, const float* __restrict__ rot,
                                                  GroupCams gc, double eps2d, const float* acc_, int astride,
                                                  int max_slots, const int32_t* gid_of_, const int32_t* n_slots_,
                                                  double* pmat_, int32_t* slot_of_, size_t vs) {
  const DevCam cam = gc.c[blockIdx.y];
  const float* __restrict__ acc = vp(acc_, vs);
  const int32_t* __restrict__ gid_of = vp(gid_of_, vs);
  double* __restrict__ pmat = vp(pmat_, vs);
  const int used = min(*vp(n_slots_, vs), max_slots);
  int32_t* __restrict__ slot_of = vp(slot_of_, vs);
  for (int slot = blockIdx.x * blockDim.x + threadIdx.x; slot < used; slot += gridDim.x * blockDim.x) {
    slot_of[gid_of[slot]] = -1;  // unslotted again for the next view (the back pass has run)
    const float a2f = acc[(size_t)slot * astride + kStatYd + tri_idx(6, 6, 7)];
    if (!(a2f > 0.f)) continue;
    double P[7][kNGeo];
    chain_rule(mean, log_scale, rot, n, gid_of[slot], cam, eps2d, P);
    double* dst = pmat + (size_t)slot * 7 * kNGeo;
    for (int i = 0; i < 7; ++i)
      for (int j = 0; j < kNGeo; ++j) dst[i * kNGeo + j] = P[i][j];
  }
}

// TRACE: the trace criterion (reductions of trace(H^-1)); else log-det gains.
template <bool TRACE>
__global__ __launch_bounds__(kFinThreads) void k_finalize(
    int n, int k, const float* __restrict__ mean, const float* __restrict__ log_scale, const float* __restrict__ rot,
    const float* __restrict__ conf, const float* __restrict__ prob, double eps2d, double lambda, uint32_t outputs,
    int mode, int conf_on_train, int criterion, const float* acc_, int astride, int max_slots, const int32_t* gid_of_,
    const int32_t* n_slots_, const int32_t* overflow_, ngs_hessian h, int has_h, double* ig_out_,
    int64_t* __restrict__ stats, int32_t* __restrict__ sticky, const double* pmat_, size_t vs) {
  __shared__ FinShared S;
  // view blockIdx.y of the group: its workspace vs bytes on, its three gains after the
  // previous views' (scoring only: accumulation into the store runs one view per launch)
  const float* __restrict__ acc = vp(acc_, vs);
  const int32_t* __restrict__ gid_of = vp(gid_of_, vs);
  const int32_t* __restrict__ overflow = vp(overflow_, vs);
  const double* __restrict__ pmat = vp(pmat_, vs);
  double* __restrict__ ig_out = ig_out_ + 3 * (size_t)blockIdx.y;
  const int used = min(*vp(n_slots_, vs), max_slots);
  if (blockIdx.x == 0 && threadIdx.x == 0 && *overflow) {
    if (stats) atomicAdd((unsigned long long*)&stats[5], 1ull);
    if (sticky) atomicOr(sticky, 1);
  }
  const int nst = stat_len(k);
  for (int slot = blockIdx.x; slot < used; slot += gridDim.x) {
    // a Gaussian that reached a tile but no pixel has no statistics (sum a^2 = 0): its gain
    // is zero and its row is not read
    const float a2f = acc[(size_t)slot * astride + kStatYd + tri_idx(6, 6, 7)];
    if (!(a2f > 0.f)) continue;
    __syncthreads();
    const int g = gid_of[slot];
    for (int s = threadIdx.x; s < nst; s += kFinThreads) S.st[s] = (double)acc[(size_t)slot * astride + s];
    __syncthreads();
    const double a2 = S.st[kStatYd + tri_idx(6, 6, 7)];
    for (int e = threadIdx.x; e < 7 * kNGeo; e += kFinThreads) S.P[e / kNGeo][e % kNGeo] = pmat[(size_t)slot * 7 * kNGeo + e];
    if (threadIdx.x == 0) {
      if (stats) atomicAdd((unsigned long long*)&stats[2], 1ull);
      S.hs = has_h ? h.slot_of[g] : -1;
      S.hs_new = 0;
    }
    for (int c = threadIdx.x; c < k; c += kFinThreads) S.p[c] = (double)prob[(size_t)g * k + c];
    __syncthreads();
    const double cg = (double)conf[g];
    const double wacc = conf_on_train ? cg : 1.0;
    if (mode == NGS_MODE_ACCUMULATE) {
      if (threadIdx.x == 0 && S.hs < 0) {
        const int ns = atomicAdd(h.n_slots, 1);
        if (ns < h.capacity) { h.slot_of[g] = ns; h.gid_of[ns] = g; S.hs = ns; S.hs_new = 1; }
      }
      __syncthreads();
      if (S.hs < 0) continue;  // store full: ngs_hessian_finalize reports it
    }
    const int hs = S.hs;
    const bool fresh = S.hs_new != 0;
    // weight of this view's block, and whether a stored H_T is added
    const double wv = mode == NGS_MODE_ACCUMULATE ? wacc : cg;
    const bool stored = mode == NGS_MODE_ACCUMULATE ? !fresh : hs >= 0;
    for (int f = 0; f < 3; ++f) {
      if (!((outputs >> f) & 1u)) continue;
      const int sl = store_len(f, k);
      double* hblk = (f == 0 ? h.h_rgb : (f == 1 ? h.h_d : h.h_o)) + (size_t)(hs < 0 ? 0 : hs) * sl;
      double ld_m;
      if (f < 2) {
        const int l = block_dim(f);
        const int tl = tri_len(l);
        // ---- the upper triangle of A (unweighted) ----
        for (int e = threadIdx.x; e < tl; e += kFinThreads) S.A[e] = 0.0;
        __syncthreads();
        if (f == 0) {
          load_sym(S, kStatYrgb, 6);
          geo_block(S, 6, l);
          for (int e = threadIdx.x; e < kNGeo * 3; e += kFinThreads) {
            const int i = e / 3, ch = e % 3;
            double v = 0.0;
            for (int a = 0; a < 6; ++a) v += S.P[a][i] * S.st[kStatXrgb + a * 3 + ch];
            S.A[tri_idx(i, kNGeo + ch, l)] = v;
          }
          if (threadIdx.x < 3) S.A[tri_idx(kNGeo + threadIdx.x, kNGeo + threadIdx.x, l)] = a2;
        } else {
          load_sym(S, kStatYd, 7);
          geo_block(S, 7, l);
        }
        __syncthreads();
        // M = (stored H_T or lambda I) + w A
        for (int e = threadIdx.x; e < tl; e += kFinThreads) S.A[e] = (stored ? hblk[e] : 0.0) + wv * S.A[e];
        __syncthreads();
        if (!stored)
          for (int i = threadIdx.x; i < l; i += kFinThreads) S.A[tri_idx(i, i, l)] += lambda;
        __syncthreads();
        if (mode == NGS_MODE_ACCUMULATE) {
          for (int e = threadIdx.x; e < tl; e += kFinThreads) hblk[e] = S.A[e];
          continue;
        }
        if constexpr (TRACE) ld_m = trace_inv_prod(S.A, l, nullptr, &S.F[0][0]);
        else ld_m = ldl_logdet<kSmallL>(S.A, l, S.row);
      } else {
        // ---- object block as (G, E, tau) ----
        load_sym(S, kStatYo, 6);
        for (int e = threadIdx.x; e < 6 * kNGeo; e += kFinThreads) {
          const int a = e / kNGeo, j = e % kNGeo;
          double v = 0.0;
          for (int b = 0; b < 6; ++b) v += S.Y[a][b] * S.P[b][j];
          S.YP[a][j] = v;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kNGeo * kNGeo; e += kFinThreads) {
          const int i = e / kNGeo, c = e % kNGeo;
          if (c < i) continue;
          double v = 0.0;
          for (int a = 0; a < 6; ++a) v += S.P[a][i] * S.YP[a][c];
          const double base = stored ? hblk[tri_idx(i, c, kNGeo)] : (i == c ? lambda : 0.0);
          v = base + wv * v;
          S.G[i][c] = v;
          S.G[c][i] = v;
        }
        // E = P^T (m1 p^T - Z_o)
        for (int e = threadIdx.x; e < kNGeo * k; e += kFinThreads) {
          const int r = e / k, c = e % k;
          double v = 0.0;
          for (int a = 0; a < 6; ++a) v += S.P[a][r] * (S.st[kStatM1 + a] * S.p[c] - S.st[kStatScalar + a * k + c]);
          S.E[r][c] = (stored ? hblk[kObjE + r * k + c] : 0.0) + wv * v;
        }
        if (threadIdx.x == 0) S.tau = (stored ? hblk[kObjTau] : 0.0) + wv * a2;
        __syncthreads();
        if (mode == NGS_MODE_ACCUMULATE) {
          for (int e = threadIdx.x; e < kNGeo * kNGeo; e += kFinThreads) {
            const int i = e / kNGeo, c = e % kNGeo;
            if (c >= i) hblk[tri_idx(i, c, kNGeo)] = S.G[i][c];
          }
          for (int e = threadIdx.x; e < kNGeo * k; e += kFinThreads) hblk[kObjE + e] = S.E[e / k][e % k];
          if (threadIdx.x == 0) {
            hblk[kObjTau] = S.tau;
            hblk[kObjLam] = lambda;
          }
          if (fresh)
            for (int c = threadIdx.x; c < k; c += kFinThreads) hblk[kObjE + kNGeo * k + c] = S.p[c];
          continue;
        }
        if constexpr (TRACE) {
          double ld_d, trd;
          object_schur(S, k, lambda, S.tau, &ld_d, &trd);
          ld_m = object_trinv_after_schur(S, k, trd);
        } else {
          ld_m = object_logdet(S, k, lambda, S.tau);
        }
      }
      // ---- SCORE: gain = logdet M - logdet H_T, or (trace criterion) the reduction of the
      // covariance trace, trace(H_T^-1) - trace(M^-1) ----
      const int l = f == 2 ? kNGeo + k : block_dim(f);
      if constexpr (TRACE) {
        const double tr_h = hs >= 0 ? h.trinv[(size_t)f * h.capacity + hs] : (double)l / lambda;
        if (threadIdx.x == 0 && cg != 0.0) atomicAdd(&ig_out[f], tr_h - ld_m);
      } else {
        const double ld_h = hs >= 0 ? h.logdet[(size_t)f * h.capacity + hs] : (double)l * log(lambda);
        if (threadIdx.x == 0 && cg != 0.0) atomicAdd(&ig_out[f], ld_m - ld_h);
      }
    }
  }
}

// logdet of every stored block (after the last training view).
__global__ __launch_bounds__(kFinThreads) void k_hessian_logdet(ngs_hessian h, int used) {
  __shared__ FinShared S;
  const int k = h.k;
  for (int slot = blockIdx.x; slot < used; slot += gridDim.x) {
    for (int f = 0; f < 3; ++f) {
      const int sl = store_len(f, k);
      const double* hblk = (f == 0 ? h.h_rgb : (f == 1 ? h.h_d : h.h_o)) + (size_t)slot * sl;
      __syncthreads();
      double ld;
      if (f < 2) {
        for (int e = threadIdx.x; e < tri_len(block_dim(f)); e += kFinThreads) S.A[e] = hblk[e];
        __syncthreads();
        ld = ldl_logdet<kSmallL>(S.A, block_dim(f), S.row);
        if (h.trinv) {
          const double tr = trace_inv_prod(S.A, block_dim(f), nullptr, &S.F[0][0]);
          if (threadIdx.x == 0) h.trinv[(size_t)f * h.capacity + slot] = tr;
        }
      } else {
        for (int e = threadIdx.x; e < kNGeo * kNGeo; e += kFinThreads) {
          const int i = e / kNGeo, c = e % kNGeo;
          S.G[i][c] = hblk[tri_idx(min(i, c), max(i, c), kNGeo)];
        }
        for (int e = threadIdx.x; e < kNGeo * k; e += kFinThreads) S.E[e / k][e % k] = hblk[kObjE + e];
        for (int c = threadIdx.x; c < k; c += kFinThreads) S.p[c] = hblk[kObjE + kNGeo * k + c];
        __syncthreads();
        double ld_d, trd;
        object_schur(S, k, hblk[kObjLam], hblk[kObjTau], &ld_d, h.trinv ? &trd : nullptr);
        ld = ld_d + ldl_logdet<kSmallL>(S.A, kNGeo, S.row);
        if (h.trinv) {
          const double tr = object_trinv_after_schur(S, k, trd);
          if (threadIdx.x == 0) h.trinv[(size_t)f * h.capacity + slot] = tr;
        }
      }
      if (threadIdx.x == 0) h.logdet[(size_t)f * h.capacity + slot] = ld;
    }
  }
}

// Eq. 10 normalisation, Eq. 11 combination and the argmax of Eq. 5 (lowest index on ties).
// The normalisers come from nf_dev (device, three doubles) when it is given, else by value.
// With the trace criterion the raw values are covariance-trace reductions R, turned into the
// set function's difference 1 / (S - R) - 1 / S = R / (S (S - R)) with the training totals S.
__global__ __launch_bounds__(256) void k_combine(const double* __restrict__ ig_raw, int nv, double n0, double n1,
                                                 double n2, const double* __restrict__ nf_dev, double bd, double bo,
                                                 uint32_t outputs, int criterion, double st0, double st1, double st2,
                                                 float* __restrict__ scores, int32_t* __restrict__ best) {
  __shared__ double sv[256];
  __shared__ int si[256];
  double bv = -INFINITY;
  int bi = -1;
  const double nf[3] = {nf_dev ? nf_dev[0] : n0, nf_dev ? nf_dev[1] : n1, nf_dev ? nf_dev[2] : n2};
  const double beta[3] = {1.0, bd, bo};
  const double st[3] = {st0, st1, st2};
  for (int v = threadIdx.x; v < nv; v += 256) {
    double tot = 0.0;
    for (int f = 0; f < 3; ++f) {
      const double r = ig_raw[3 * v + f];
      const double g = criterion == 1 ? r / (st[f] * (st[f] - r)) : r;
      const double s = ((outputs >> f) & 1u) ? g / nf[f] : 0.0;
      scores[4 * v + f] = (float)s;
      tot += beta[f] * s;
    }
    scores[4 * v + 3] = (float)tot;
    if (tot > bv) { bv = tot; bi = v; }
  }
  sv[threadIdx.x] = bv;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      const double ov = sv[threadIdx.x + off];
      const int oi = si[threadIdx.x + off];
      if (oi >= 0 && (si[threadIdx.x] < 0 || ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi < si[threadIdx.x]))) {
        sv[threadIdx.x] = ov;
        si[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *best = si[0];
}

}  // namespace

hipError_t launch_ig_finalize(const ngs_scene& s, const Group& G, const ngs_raster_params& rp, const ngs_ig_params& ig,
                              const IgWs& w, ngs_hessian* h, double* ig_out, int64_t* stats, int32_t* sticky,
                              hipStream_t st) {
  // accumulation writes the shared store: two views of one launch would race on a slot
  if (ig.mode == NGS_MODE_ACCUMULATE && G.g != 1) return hipErrorInvalidValue;
  ngs_hessian hh{};
  if (h) hh = *h;
  const int blocks = (int)std::min<int64_t>(w.max_slots, std::max(512, 4096 / G.g));
  const int cblocks = (int)std::min<int64_t>((w.max_slots + 63) / 64, std::max(256, 2048 / G.g));
  ProfScope ps(kProfIgFinalize, st);
  hipLaunchKernelGGL(k_fin_chain, dim3(cblocks, G.g), dim3(64), 0, st, s.n, s.mean, s.log_scale, s.rot, G.cams,
                     (double)rp.eps2d, w.acc, w.astride, (int)w.max_slots, w.gid_of, w.n_slots, w.pmat, w.slot_of,
                     G.vs);
  auto fin = ig.criterion == 1 ? k_finalize<true> : k_finalize<false>;
  hipLaunchKernelGGL(fin, dim3(blocks, G.g), dim3(kFinThreads), 0, st, s.n, s.k, s.mean, s.log_scale, s.rot, s.conf,
                     s.prob, (double)rp.eps2d, (double)ig.lambda_prior, ig.outputs, ig.mode, ig.conf_on_train,
                     ig.criterion, w.acc, w.astride, (int)w.max_slots, w.gid_of, w.n_slots, w.overflow, hh, h ? 1 : 0,
                     ig_out, stats, sticky, (const double*)w.pmat, G.vs);
  return hipGetLastError();
}

// Eq. 10 normalisers of the training set: n_f = mean over the training views t of IG_f(T, t).
// For the trace-based f (Sec. III-B) the per-view quantity is the set-function gain
// f(T + t) - f(T) = R / (S (S - R)) of the raw trace reduction R, where S_f = sum over every
// Gaussian of trace(H_T,g^-1): the stored slots' traces plus l_f / lambda for each of the
// other n - used Gaussians (H_T = lambda I). One block; the slot sum runs in a fixed order.
__global__ __launch_bounds__(256) void k_train_norm(const double* __restrict__ trinv, const int32_t* __restrict__ n_slots,
                                                     int capacity, int n, int k, double lambda, int criterion,
                                                     const double* __restrict__ ig_train, int n_train,
                                                     double* __restrict__ norm, double* __restrict__ trace_total) {
  __shared__ double sm[3][256];
  const int used = trinv ? min(*n_slots, capacity) : 0;
  double acc[3] = {0.0, 0.0, 0.0};
  if (criterion == 1 && trinv)
    for (int s = threadIdx.x; s < used; s += 256)
      for (int f = 0; f < 3; ++f) acc[f] += trinv[(size_t)f * capacity + s];
  for (int f = 0; f < 3; ++f) sm[f][threadIdx.x] = acc[f];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int f = 0; f < 3; ++f) sm[f][threadIdx.x] += sm[f][threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double dims[3] = {14.0, 11.0, 11.0 + (double)k};
  for (int f = 0; f < 3; ++f) {
    const double S = criterion == 1 ? sm[f][0] + (double)(n - used) * dims[f] / lambda : 0.0;
    double mean = 0.0;
    for (int t = 0; t < n_train; ++t) {
      const double r = ig_train[3 * t + f];
      mean += criterion == 1 ? r / (S * (S - r)) : r;
    }
    norm[f] = n_train > 0 ? mean / (double)n_train : 0.0;
    if (trace_total) trace_total[f] = S;
  }
}

hipError_t launch_train_normalisers(const ngs_hessian& h, int n, int k, const ngs_ig_params& ig, const double* ig_train,
                                    int n_train, double* norm, double* trace_total, hipStream_t st) {
  ProfScope ps(kProfCombine, st);
  hipLaunchKernelGGL(k_train_norm, dim3(1), dim3(256), 0, st, ig.criterion == 1 ? h.trinv : nullptr, h.n_slots,
                     h.capacity, n, k, (double)ig.lambda_prior, ig.criterion, ig_train, n_train, norm, trace_total);
  return hipGetLastError();
}

hipError_t launch_hessian_logdet(ngs_hessian* h, int32_t n_slots, float lambda_prior, hipStream_t st) {
  const int used = std::min(n_slots, h->capacity);
  if (used <= 0) return hipSuccess;
  ProfScope ps(kProfHessianLogdet, st);
  hipLaunchKernelGGL(k_hessian_logdet, dim3(std::min(used, 4096)), dim3(kFinThreads), 0, st, *h, used);
  (void)lambda_prior;
  return hipGetLastError();
}

hipError_t launch_score_combine(const double* ig_raw, int n_views, double n0, double n1, double n2,
                                const double* nf_dev, const ngs_ig_params& ig, float* scores, int32_t* best,
                                hipStream_t st) {
  ProfScope ps(kProfCombine, st);
  hipLaunchKernelGGL(k_combine, dim3(1), dim3(256), 0, st, ig_raw, n_views, n0, n1, n2, nf_dev, (double)ig.beta_d,
                     (double)ig.beta_o, ig.outputs, ig.criterion, ig.trace_total[0], ig.trace_total[1],
                     ig.trace_total[2], scores, best);
  return hipGetLastError();
}

}  // namespace ngs
