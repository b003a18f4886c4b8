// ngs_oracle.cpp -- plain, slow FP64 CPU oracle for object-aware next-best-view scoring.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or calls this
// file; only the tests, the smoke check and the benchmark's CPU-baseline leg do.
// It shares no source with the HIP path: different algorithm (dense parameter-space
// Jacobian rows and dense per-Gaussian blocks), different precision (FP64 throughout),
// different derivative machinery (forward-mode dual numbers instead of a hand chain rule).
//
// What it computes, and where each step comes from in arXiv 2602.08266:
//   * per-Gaussian object probability p = softmax(o) (Sec. III-A.1, after Eq. 3),
//     confidence c_g (Eq. 7; object-centric variant Eq. 12);
//   * projection and tile binning of the 3DGS pipeline the paper follows (Sec. IV-A.2:
//     "follows the original 3DGS pipeline");
//   * front-to-back compositing of colour, depth and the object vector (Eq. 1) with the
//     background residual (Eq. 2);
//   * Jacobian rows of every rendered channel w.r.t. the raw Gaussian parameters, the
//     Gauss-Newton information J^T J per view (Eq. 6), kept block-diagonal per Gaussian
//     (Sec. III-B.1) and confidence-weighted (Eqs. 8-9), with per-output parameter subsets
//     (Sec. III-B.3: all outputs use position, scale, rotation, opacity; RGB adds colour,
//     masks add the object vector);
//   * information gain as a log-det difference (Eqs. 5-6), per-output normalisation by the
//     training-view mean (Eq. 10), weighted combination (Eq. 11), argmax (Eq. 5).
// Readings where the paper is silent (prior lambda*I, rasterizer constants, parameterisation,
// depth definition, tie-breaks) are parameters here and are listed in the design notes.
//
// Build: g++ -O2 -std=c++17 -ffp-contract=off -shared -fPIC -pthread (no FMA contraction,
// so that the FP64 projection is evaluated exactly in the written order).

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

namespace {

constexpr int NGEO = 11;  // mu(3), log-scale(3), raw quaternion(4), opacity logit(1)

// ----------------------------------------------------------------------------------------
// Forward-mode dual numbers with NGEO infinitesimal directions.
// ----------------------------------------------------------------------------------------
struct Dual {
  double v;
  double d[NGEO];
  Dual() : v(0) { std::memset(d, 0, sizeof d); }
  explicit Dual(double x) : v(x) { std::memset(d, 0, sizeof d); }
  static Dual var(double x, int i) { Dual r(x); r.d[i] = 1.0; return r; }
};
inline Dual operator+(const Dual& a, const Dual& b) { Dual r; r.v = a.v + b.v; for (int i = 0; i < NGEO; ++i) r.d[i] = a.d[i] + b.d[i]; return r; }
inline Dual operator-(const Dual& a, const Dual& b) { Dual r; r.v = a.v - b.v; for (int i = 0; i < NGEO; ++i) r.d[i] = a.d[i] - b.d[i]; return r; }
inline Dual operator-(const Dual& a) { Dual r; r.v = -a.v; for (int i = 0; i < NGEO; ++i) r.d[i] = -a.d[i]; return r; }
inline Dual operator*(const Dual& a, const Dual& b) { Dual r; r.v = a.v * b.v; for (int i = 0; i < NGEO; ++i) r.d[i] = a.d[i] * b.v + a.v * b.d[i]; return r; }
inline Dual operator*(double s, const Dual& a) { Dual r; r.v = s * a.v; for (int i = 0; i < NGEO; ++i) r.d[i] = s * a.d[i]; return r; }
inline Dual operator+(double s, const Dual& a) { Dual r = a; r.v = s + a.v; return r; }
inline Dual operator-(double s, const Dual& a) { Dual r = -a; r.v = s - a.v; return r; }
inline Dual operator/(const Dual& a, const Dual& b) {
  Dual r; r.v = a.v / b.v;
  for (int i = 0; i < NGEO; ++i) r.d[i] = (a.d[i] * b.v - a.v * b.d[i]) / (b.v * b.v);
  return r;
}
inline Dual dexp(const Dual& a) { Dual r; r.v = std::exp(a.v); for (int i = 0; i < NGEO; ++i) r.d[i] = r.v * a.d[i]; return r; }
inline Dual dsqrt(const Dual& a) { Dual r; r.v = std::sqrt(a.v); for (int i = 0; i < NGEO; ++i) r.d[i] = a.d[i] / (2.0 * r.v); return r; }

}  // namespace

extern "C" {

// Scene, structure of arrays, FP64 copies of the float32 inputs.
struct or_scene {
  int32_t n, k;
  const double* mean;           // [3][n]
  const double* log_scale;      // [3][n]
  const double* rot;            // [4][n] raw quaternion (w, x, y, z)
  const double* opacity_logit;  // [n]
  const double* rgb;            // [3][n]
  const double* obj_logit;      // [k][n]
};
// Pinhole camera, world -> camera rotation R (row-major) and translation t.
struct or_camera {
  double R[9], t[3], fx, fy, cx, cy;
  int32_t width, height;
};
struct or_raster {
  int32_t tile;
  double z_near, eps2d, cutoff_q, alpha_min, alpha_max, t_min, amb_rel;
};
struct or_ig {
  double lambda_prior, alpha_obj, alpha_opa, beta_d, beta_o;
  int32_t target_id;      // -1: whole scene (Eq. 7); else the object id of Eq. 12
  int32_t outputs;        // bit 0 rgb, bit 1 depth, bit 2 object
  int32_t conf_on_train;  // 1: H_T = lambda I + c_g sum_t A_t; 0: H_T = lambda I + sum_t A_t
  int32_t obj_eq2;        // 1: object output is O (Eq. 2); 0: O' (Eq. 1)
  int32_t level;          // 1: dense object rows; 2: block expansion of the object rows
  int32_t criterion;      // 0: f = log det H (Eq. 6); 1: f = trace(H^-1)^-1 (Sec. III-B)
};

}  // extern "C"

namespace {

// ----------------------------------------------------------------------------------------
// Per-Gaussian terms: sigma = sigmoid(l), p = softmax(o), kappa = max_k p, argmax, c_g.
// ----------------------------------------------------------------------------------------
struct GaussTerms {
  std::vector<double> p, kappa, sigma, conf;
  std::vector<int32_t> amax;
};

GaussTerms gaussian_terms(const or_scene& s, const or_ig& ig) {
  GaussTerms gt;
  const int n = s.n, k = s.k;
  gt.p.assign((size_t)n * k, 0.0);
  gt.kappa.assign(n, 0.0);
  gt.sigma.assign(n, 0.0);
  gt.conf.assign(n, 0.0);
  gt.amax.assign(n, 0);
  for (int g = 0; g < n; ++g) {
    double mx = -INFINITY;
    for (int c = 0; c < k; ++c) mx = std::max(mx, s.obj_logit[(size_t)c * n + g]);
    double z = 0.0;
    for (int c = 0; c < k; ++c) z += std::exp(s.obj_logit[(size_t)c * n + g] - mx);
    int am = 0;
    for (int c = 0; c < k; ++c) {
      double pc = std::exp(s.obj_logit[(size_t)c * n + g] - mx) / z;
      gt.p[(size_t)g * k + c] = pc;
      if (pc > gt.p[(size_t)g * k + am]) am = c;  // lowest index on ties
    }
    gt.amax[g] = am;
    gt.kappa[g] = gt.p[(size_t)g * k + am];
    gt.sigma[g] = 1.0 / (1.0 + std::exp(-s.opacity_logit[g]));
    if (ig.target_id < 0) {
      // Eq. 7: c_g = (max_k p_gk)^(-alpha_obj) * sigma_g^(-alpha_opa)
      gt.conf[g] = std::pow(gt.kappa[g], -ig.alpha_obj) * std::pow(gt.sigma[g], -ig.alpha_opa);
    } else {
      // Eq. 12: target probability instead of the maximum; zero off the target object.
      const int obj = ig.target_id;
      gt.conf[g] = (am == obj) ? std::pow(gt.p[(size_t)g * k + obj], -ig.alpha_obj) *
                                     std::pow(gt.sigma[g], -ig.alpha_opa)
                               : 0.0;
    }
  }
  return gt;
}

// ----------------------------------------------------------------------------------------
// Projection (value path, FP64, written order, no contraction).
// ----------------------------------------------------------------------------------------
struct Proj {
  double z, mx, my;
  double cov[3];    // Sigma2 (a, b, c) incl. eps
  double conic[3];  // Q = Sigma2^-1 (xx, xy, yy)
  int32_t radius;
  int32_t rect[4];  // x0, y0, x1, y1 (inclusive tiles)
  uint32_t zkey;    // bits of float32(Z)
  bool in_front;    // Z > z_near
  bool valid;       // in front and the tile rect is not empty
};

void quat_to_rot(double w, double x, double y, double z, double Rg[9]) {
  Rg[0] = 1.0 - 2.0 * (y * y + z * z); Rg[1] = 2.0 * (x * y - w * z);       Rg[2] = 2.0 * (x * z + w * y);
  Rg[3] = 2.0 * (x * y + w * z);       Rg[4] = 1.0 - 2.0 * (x * x + z * z); Rg[5] = 2.0 * (y * z - w * x);
  Rg[6] = 2.0 * (x * z - w * y);       Rg[7] = 2.0 * (y * z + w * x);       Rg[8] = 1.0 - 2.0 * (x * x + y * y);
}

Proj project_one(const or_scene& s, int g, const or_camera& cam, const or_raster& rp) {
  const int n = s.n;
  Proj P{};
  const double mu[3] = {s.mean[g], s.mean[n + g], s.mean[2 * n + g]};
  double X[3];
  for (int i = 0; i < 3; ++i)
    X[i] = ((cam.R[3 * i] * mu[0] + cam.R[3 * i + 1] * mu[1]) + cam.R[3 * i + 2] * mu[2]) + cam.t[i];
  P.z = X[2];
  P.in_front = P.z > rp.z_near;
  P.valid = false;
  if (!P.in_front) return P;
  P.mx = (cam.fx * X[0]) / P.z + cam.cx;
  P.my = (cam.fy * X[1]) / P.z + cam.cy;
  // Sigma3 = Rg diag(s^2) Rg^T
  const double sc[3] = {std::exp(s.log_scale[g]), std::exp(s.log_scale[n + g]), std::exp(s.log_scale[2 * n + g])};
  const double qw = s.rot[g], qx = s.rot[n + g], qy = s.rot[2 * n + g], qz = s.rot[3 * n + g];
  const double qn = std::sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
  double Rg[9];
  quat_to_rot(qw / qn, qx / qn, qy / qn, qz / qn, Rg);
  double S3[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0.0;
      for (int k = 0; k < 3; ++k) acc = acc + (Rg[3 * i + k] * (sc[k] * sc[k])) * Rg[3 * j + k];
      S3[3 * i + j] = acc;
    }
  // Perspective Jacobian of (fx X/Z + cx, fy Y/Z + cy) at X.
  const double Jp[6] = {cam.fx / P.z, 0.0, -(cam.fx * X[0]) / (P.z * P.z),
                        0.0, cam.fy / P.z, -(cam.fy * X[1]) / (P.z * P.z)};
  double T[6];  // Jp * R (2x3)
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j)
      T[3 * i + j] = ((Jp[3 * i] * cam.R[j] + Jp[3 * i + 1] * cam.R[3 + j]) + Jp[3 * i + 2] * cam.R[6 + j]);
  double M[6];  // T * Sigma3 (2x3)
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j)
      M[3 * i + j] = ((T[3 * i] * S3[j] + T[3 * i + 1] * S3[3 + j]) + T[3 * i + 2] * S3[6 + j]);
  double S2[4];  // M * T^T (2x2)
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      S2[2 * i + j] = ((M[3 * i] * T[3 * j] + M[3 * i + 1] * T[3 * j + 1]) + M[3 * i + 2] * T[3 * j + 2]);
  const double a = S2[0] + rp.eps2d, b = S2[1], c = S2[3] + rp.eps2d;
  P.cov[0] = a; P.cov[1] = b; P.cov[2] = c;
  const double det = a * c - b * b;
  P.conic[0] = c / det; P.conic[1] = -b / det; P.conic[2] = a / det;
  const double half = (a - c) * 0.5;
  const double lmax = (a + c) * 0.5 + std::sqrt(half * half + b * b);
  const double r = std::ceil(3.0 * std::sqrt(lmax));
  P.radius = (int32_t)std::min(r, 1.0e9);
  const int TW = (cam.width + rp.tile - 1) / rp.tile, TH = (cam.height + rp.tile - 1) / rp.tile;
  auto tile_of = [&](double v, int lim) {
    double f = std::floor(v / (double)rp.tile);
    if (f < -1.0) f = -1.0;
    if (f > (double)lim) f = (double)lim;
    return (int)f;
  };
  int x0 = std::max(0, tile_of(P.mx - r, TW));
  int x1 = std::min(TW - 1, tile_of(P.mx + r, TW));
  int y0 = std::max(0, tile_of(P.my - r, TH));
  int y1 = std::min(TH - 1, tile_of(P.my + r, TH));
  P.rect[0] = x0; P.rect[1] = y0; P.rect[2] = x1; P.rect[3] = y1;
  P.valid = (x0 <= x1) && (y0 <= y1);
  const float zf = (float)P.z;
  std::memcpy(&P.zkey, &zf, 4);
  return P;
}

// Dual-number projection: (mx, my, Qxx, Qxy, Qyy, Z, sigma) as functions of the 11
// geometric parameters of one Gaussian.
struct DualProj {
  Dual mx, my, q[3], z, sigma;
};

DualProj project_dual(const or_scene& s, int g, const or_camera& cam, const or_raster& rp) {
  const int n = s.n;
  Dual mu[3], ls[3], qq[4];
  for (int i = 0; i < 3; ++i) mu[i] = Dual::var(s.mean[(size_t)i * n + g], i);
  for (int i = 0; i < 3; ++i) ls[i] = Dual::var(s.log_scale[(size_t)i * n + g], 3 + i);
  for (int i = 0; i < 4; ++i) qq[i] = Dual::var(s.rot[(size_t)i * n + g], 6 + i);
  Dual ell = Dual::var(s.opacity_logit[g], 10);
  Dual X[3];
  for (int i = 0; i < 3; ++i)
    X[i] = cam.R[3 * i] * mu[0] + cam.R[3 * i + 1] * mu[1] + cam.R[3 * i + 2] * mu[2] + Dual(cam.t[i]);
  DualProj D;
  D.z = X[2];
  D.mx = cam.fx * X[0] / X[2] + Dual(cam.cx);
  D.my = cam.fy * X[1] / X[2] + Dual(cam.cy);
  Dual sc2[3];
  for (int i = 0; i < 3; ++i) { Dual e = dexp(ls[i]); sc2[i] = e * e; }
  Dual qn = dsqrt(qq[0] * qq[0] + qq[1] * qq[1] + qq[2] * qq[2] + qq[3] * qq[3]);
  Dual w = qq[0] / qn, x = qq[1] / qn, y = qq[2] / qn, z = qq[3] / qn;
  Dual Rg[9];
  Rg[0] = 1.0 - 2.0 * (y * y + z * z); Rg[1] = 2.0 * (x * y - w * z);       Rg[2] = 2.0 * (x * z + w * y);
  Rg[3] = 2.0 * (x * y + w * z);       Rg[4] = 1.0 - 2.0 * (x * x + z * z); Rg[5] = 2.0 * (y * z - w * x);
  Rg[6] = 2.0 * (x * z - w * y);       Rg[7] = 2.0 * (y * z + w * x);       Rg[8] = 1.0 - 2.0 * (x * x + y * y);
  Dual S3[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      Dual acc(0.0);
      for (int k = 0; k < 3; ++k) acc = acc + Rg[3 * i + k] * sc2[k] * Rg[3 * j + k];
      S3[3 * i + j] = acc;
    }
  Dual Jp[6] = {cam.fx * (Dual(1.0) / X[2]), Dual(0.0), -(cam.fx * X[0] / (X[2] * X[2])),
                Dual(0.0), cam.fy * (Dual(1.0) / X[2]), -(cam.fy * X[1] / (X[2] * X[2]))};
  Dual T[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j)
      T[3 * i + j] = cam.R[j] * Jp[3 * i] + cam.R[3 + j] * Jp[3 * i + 1] + cam.R[6 + j] * Jp[3 * i + 2];
  Dual S2[4];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      Dual acc(0.0);
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) acc = acc + T[3 * i + k] * S3[3 * k + l] * T[3 * j + l];
      S2[2 * i + j] = acc;
    }
  Dual a = S2[0] + Dual(rp.eps2d), b = S2[1], c = S2[3] + Dual(rp.eps2d);
  Dual det = a * c - b * b;
  D.q[0] = c / det;
  D.q[1] = -b / det;
  D.q[2] = a / det;
  D.sigma = Dual(1.0) / (1.0 + dexp(-ell));
  return D;
}

// ----------------------------------------------------------------------------------------
// Tile lists: every (tile, Gaussian) pair of the rects, sorted by (tile, f32 depth bits, gid).
// ----------------------------------------------------------------------------------------
struct Lists {
  std::vector<uint64_t> keys;
  std::vector<uint32_t> gids;
  std::vector<uint32_t> start, end;
  int tw, th;
};

Lists build_lists(const std::vector<Proj>& pr, int width, int height, int tile) {
  Lists L;
  L.tw = (width + tile - 1) / tile;
  L.th = (height + tile - 1) / tile;
  struct E { uint32_t tile, zkey, gid; };
  std::vector<E> es;
  for (size_t g = 0; g < pr.size(); ++g) {
    const Proj& P = pr[g];
    if (!P.valid) continue;
    for (int ty = P.rect[1]; ty <= P.rect[3]; ++ty)
      for (int tx = P.rect[0]; tx <= P.rect[2]; ++tx)
        es.push_back({(uint32_t)(ty * L.tw + tx), P.zkey, (uint32_t)g});
  }
  std::sort(es.begin(), es.end(), [](const E& a, const E& b) {
    if (a.tile != b.tile) return a.tile < b.tile;
    if (a.zkey != b.zkey) return a.zkey < b.zkey;
    return a.gid < b.gid;
  });
  const int nt = L.tw * L.th;
  L.start.assign(nt, 0);
  L.end.assign(nt, 0);
  L.keys.resize(es.size());
  L.gids.resize(es.size());
  for (size_t i = 0; i < es.size(); ++i) {
    L.keys[i] = ((uint64_t)es[i].tile << 32) | es[i].zkey;
    L.gids[i] = es[i].gid;
  }
  size_t i = 0;
  for (int t = 0; t < nt; ++t) {
    L.start[t] = (uint32_t)i;
    while (i < es.size() && es[i].tile == (uint32_t)t) ++i;
    L.end[t] = (uint32_t)i;
  }
  return L;
}

// ----------------------------------------------------------------------------------------
// Per-pixel compositing (Eq. 1 with the 3DGS cut-off rules), FP64.
// ----------------------------------------------------------------------------------------
struct Contrib {
  int gid;
  double alpha, T, a, q;  // a = alpha * T (T before this Gaussian)
  bool clamped;           // alpha held at alpha_max (no derivative through alpha)
};

struct PixelWalk {
  std::vector<Contrib> c;
  double t_final;
  bool ambiguous;
};

inline bool near_rel(double v, double ref, double rel) { return std::fabs(v - ref) <= rel * std::fabs(ref); }

// Walks `order` (gids, front to back) at pixel centre (x, y).
void walk_pixel(const int* order, size_t len, double x, double y, const std::vector<Proj>& pr,
                const GaussTerms& gt, const or_raster& rp, PixelWalk& out) {
  out.c.clear();
  out.ambiguous = false;
  double T = 1.0;
  for (size_t i = 0; i < len; ++i) {
    const int g = order[i];
    const Proj& P = pr[g];
    const double dx = x - P.mx, dy = y - P.my;
    const double q = P.conic[0] * dx * dx + 2.0 * P.conic[1] * dx * dy + P.conic[2] * dy * dy;
    if (near_rel(q, rp.cutoff_q, rp.amb_rel)) out.ambiguous = true;
    if (q > rp.cutoff_q) continue;
    const double raw = gt.sigma[g] * std::exp(-0.5 * q);
    if (near_rel(raw, rp.alpha_max, rp.amb_rel) || near_rel(raw, rp.alpha_min, rp.amb_rel)) out.ambiguous = true;
    const double alpha = std::min(rp.alpha_max, raw);
    if (alpha < rp.alpha_min) continue;
    const double Tn = T * (1.0 - alpha);
    if (near_rel(Tn, rp.t_min, rp.amb_rel)) out.ambiguous = true;
    if (Tn < rp.t_min) break;  // stop before compositing this Gaussian
    out.c.push_back({g, alpha, T, alpha * T, q, raw >= rp.alpha_max});
    T = Tn;
  }
  out.t_final = T;
}

struct Features {
  // per contributor: rgb[3], z, p[k]
  const or_scene* s;
  const std::vector<Proj>* pr;
  const GaussTerms* gt;
};

// Jacobian rows of every output channel at one pixel w.r.t. contributor `ci`'s parameters.
// rgb rows: 3 x 14 (geo 11, rgb 3); depth row: 11; object rows: k x (11 + k).
struct Rows {
  int k;
  double rgb[3][14];
  double d[NGEO];
  std::vector<double> o;  // [k][11 + k]
  // factored form used by the level-2 block expansion
  double gvec[NGEO];
  std::vector<double> wo;  // d O_k / d alpha, [k]
  double a;
};

// Suffix sums S_ch(i) = sum over contributors after i of phi_ch * a, for every contributor.
struct Suffix {
  int k;
  std::vector<double> rgb, d, o;  // [nc][3], [nc], [nc][k]
};

void pixel_suffix(const PixelWalk& W, const Features& F, Suffix& S) {
  const or_scene& s = *F.s;
  const int n = s.n, k = s.k;
  const int nc = (int)W.c.size();
  S.k = k;
  S.rgb.assign((size_t)nc * 3, 0.0);
  S.d.assign(nc, 0.0);
  S.o.assign((size_t)nc * k, 0.0);
  for (int i = nc - 2; i >= 0; --i) {
    const int h = W.c[i + 1].gid;
    const double a = W.c[i + 1].a;
    for (int ch = 0; ch < 3; ++ch) S.rgb[3 * i + ch] = S.rgb[3 * (i + 1) + ch] + s.rgb[(size_t)ch * n + h] * a;
    S.d[i] = S.d[i + 1] + (*F.pr)[h].z * a;
    for (int m = 0; m < k; ++m) S.o[(size_t)i * k + m] = S.o[(size_t)(i + 1) * k + m] + F.gt->p[(size_t)h * k + m] * a;
  }
}

void pixel_rows(const PixelWalk& W, const Suffix& Sx, int ci, double x, double y, const Features& F,
                const std::vector<DualProj>& dp, const std::vector<int>& dp_index,
                const or_ig& ig, bool dense_obj, Rows& R) {
  const or_scene& s = *F.s;
  const int n = s.n, k = s.k;
  const Contrib& C = W.c[ci];
  const int g = C.gid;
  R.k = k;
  const double* Srgb = &Sx.rgb[3 * ci];
  const double Sd = Sx.d[ci];
  const double* So = &Sx.o[(size_t)ci * k];
  const double om = 1.0 - C.alpha;
  // d alpha / d theta_geo from the dual projection (zero where alpha is clamped).
  const DualProj& D = dp[dp_index[g]];
  Dual dx = Dual(x) - D.mx, dy = Dual(y) - D.my;
  Dual q = D.q[0] * dx * dx + 2.0 * (D.q[1] * dx * dy) + D.q[2] * dy * dy;
  Dual al = D.sigma * dexp(-0.5 * q);
  for (int i = 0; i < NGEO; ++i) R.gvec[i] = C.clamped ? 0.0 : al.d[i];
  R.a = C.a;
  // RGB: out_ch = sum_i rgb_i,ch a_i.
  for (int ch = 0; ch < 3; ++ch) {
    const double w = s.rgb[(size_t)ch * n + g] * C.T - Srgb[ch] / om;
    for (int i = 0; i < NGEO; ++i) R.rgb[ch][i] = w * R.gvec[i];
    for (int m = 0; m < 3; ++m) R.rgb[ch][NGEO + m] = (m == ch) ? C.a : 0.0;
  }
  // Depth: out = sum_i Z_i a_i, Z_i also depends on mu_i directly.
  {
    const double w = (*F.pr)[g].z * C.T - Sd / om;
    for (int i = 0; i < NGEO; ++i) R.d[i] = w * R.gvec[i] + C.a * D.z.d[i];
  }
  // Object vector: O'_k = sum_i p_i,k a_i; O_0 += T_final (Eq. 2).
  if (dense_obj) R.o.assign((size_t)k * (NGEO + k), 0.0);
  R.wo.assign(k, 0.0);
  const double* pg = &F.gt->p[(size_t)g * k];
  for (int m = 0; m < k; ++m) {
    double w = pg[m] * C.T - So[m] / om;
    if (m == 0 && ig.obj_eq2) w -= W.t_final / om;
    R.wo[m] = w;
    if (!dense_obj) continue;
    double* row = &R.o[(size_t)m * (NGEO + k)];
    for (int i = 0; i < NGEO; ++i) row[i] = w * R.gvec[i];
    for (int j = 0; j < k; ++j) row[NGEO + j] = C.a * pg[m] * ((m == j ? 1.0 : 0.0) - pg[j]);
  }
}

// Dense per-Gaussian information blocks A^f_g = sum_pixels sum_ch J J^T (Eq. 6, block diagonal).
struct Blocks {
  std::vector<double> rgb, d, o;  // 14x14, 11x11, (11+k)x(11+k), full square
  double a2 = 0.0;                // level 2: pending sum of a^2 for the a^2 S S term
};

struct BlockMap {
  int k;
  std::vector<int> order;  // gids in first-touch order
  std::unordered_map<int, Blocks> m;
  Blocks& get(int g) {
    auto it = m.find(g);
    if (it != m.end()) return it->second;
    Blocks& b = m[g];
    const int lo = NGEO + k;
    b.rgb.assign(14 * 14, 0.0);
    b.d.assign(NGEO * NGEO, 0.0);
    b.o.assign((size_t)lo * lo, 0.0);
    order.push_back(g);
    return b;
  }
};

void add_outer(double* A, const double* r, int l, double wgt = 1.0) {
  for (int i = 0; i < l; ++i) {
    const double ri = r[i] * wgt;
    for (int j = 0; j < l; ++j) A[(size_t)i * l + j] += ri * r[j];
  }
}

void accumulate_rows(const Rows& R, const double* pg, int level, Blocks& B) {
  const int k = R.k, lo = NGEO + k;
  for (int ch = 0; ch < 3; ++ch) add_outer(B.rgb.data(), R.rgb[ch], 14);
  add_outer(B.d.data(), R.d, NGEO);
  if (level == 1) {
    for (int m = 0; m < k; ++m) add_outer(B.o.data(), &R.o[(size_t)m * lo], lo);
    return;
  }
  // Level 2: sum_k J_k^T J_k = [[|w|^2 g g^T, a g (S w)^T], [a (S w) g^T, a^2 S S]],
  // S = diag(p) - p p^T (softmax Jacobian), w = d O / d alpha.
  double w2 = 0.0;
  for (int m = 0; m < k; ++m) w2 += R.wo[m] * R.wo[m];
  double pw = 0.0;
  for (int m = 0; m < k; ++m) pw += pg[m] * R.wo[m];
  std::vector<double> Sw(k);
  for (int m = 0; m < k; ++m) Sw[m] = pg[m] * R.wo[m] - pg[m] * pw;
  double* A = B.o.data();
  for (int i = 0; i < NGEO; ++i)
    for (int j = 0; j < NGEO; ++j) A[(size_t)i * lo + j] += w2 * R.gvec[i] * R.gvec[j];
  for (int i = 0; i < NGEO; ++i)
    for (int m = 0; m < k; ++m) {
      const double v = R.a * R.gvec[i] * Sw[m];
      A[(size_t)i * lo + NGEO + m] += v;
      A[(size_t)(NGEO + m) * lo + i] += v;
    }
  // a^2 S S: S is constant per Gaussian, so only sum_pixels a^2 is accumulated here.
  B.a2 += R.a * R.a;
}

// Adds (sum a^2) S S to the object block of a level-2 accumulation.
void finish_level2(Blocks& B, const double* pg, int k) {
  const int lo = NGEO + k;
  std::vector<double> S((size_t)k * k);
  for (int m = 0; m < k; ++m)
    for (int j = 0; j < k; ++j) S[(size_t)m * k + j] = pg[m] * ((m == j ? 1.0 : 0.0) - pg[j]);
  for (int m = 0; m < k; ++m)
    for (int j = 0; j < k; ++j) {
      double ss = 0.0;
      for (int l = 0; l < k; ++l) ss += S[(size_t)m * k + l] * S[(size_t)l * k + j];
      B.o[(size_t)(NGEO + m) * lo + NGEO + j] += B.a2 * ss;
    }
  B.a2 = 0.0;
}

// ----------------------------------------------------------------------------------------
// One view: projection, lists, per-pixel walks; optional images and blocks.
// ----------------------------------------------------------------------------------------
struct ViewCtx {
  ViewCtx(const or_scene* s_, const or_camera* c_, const or_raster* r_, const or_ig* i_, const GaussTerms* g_)
      : s(s_), cam(c_), rp(r_), ig(i_), gt(g_) {}
  const or_scene* s;
  const or_camera* cam;
  const or_raster* rp;
  const or_ig* ig;
  const GaussTerms* gt;
  std::vector<Proj> pr;
  Lists L;
  std::vector<int> brute;  // all in-front Gaussians sorted by (zkey, gid)
};

void view_setup(ViewCtx& V) {
  const int n = V.s->n;
  V.pr.resize(n);
  for (int g = 0; g < n; ++g) V.pr[g] = project_one(*V.s, g, *V.cam, *V.rp);
  V.L = build_lists(V.pr, V.cam->width, V.cam->height, V.rp->tile);
}

void build_brute(ViewCtx& V) {
  V.brute.clear();
  for (int g = 0; g < V.s->n; ++g)
    if (V.pr[g].in_front) V.brute.push_back(g);
  std::sort(V.brute.begin(), V.brute.end(), [&](int a, int b) {
    if (V.pr[a].zkey != V.pr[b].zkey) return V.pr[a].zkey < V.pr[b].zkey;
    return a < b;
  });
}

struct BlocksResult {
  int k;
  std::vector<int> gids;  // ascending
  std::vector<Blocks> blocks;
  int64_t pairs = 0;
};

// Accumulates the blocks of one view; tiles are split into rows processed in parallel,
// each row with its own map, merged in row order (deterministic for any thread count).
BlocksResult view_blocks(ViewCtx& V, int threads) {
  const or_scene& s = *V.s;
  const int k = s.k, n = s.n;
  const int tile = V.rp->tile;
  const int W = V.cam->width, H = V.cam->height;
  // dual projections for every valid Gaussian
  std::vector<int> dp_index(n, -1);
  std::vector<int> valid_ids;
  for (int g = 0; g < n; ++g)
    if (V.pr[g].valid) { dp_index[g] = (int)valid_ids.size(); valid_ids.push_back(g); }
  std::vector<DualProj> dp(valid_ids.size());
  Features F{V.s, &V.pr, V.gt};
  auto work_dual = [&](int t0, int t1) {
    for (int i = t0; i < t1; ++i) dp[i] = project_dual(s, valid_ids[i], *V.cam, *V.rp);
  };
  threads = std::max(1, threads);
  {
    std::vector<std::thread> th;
    const int nv = (int)valid_ids.size();
    for (int t = 0; t < threads; ++t) th.emplace_back(work_dual, (int)((int64_t)nv * t / threads), (int)((int64_t)nv * (t + 1) / threads));
    for (auto& x : th) x.join();
  }
  const int nrows = V.L.th;
  std::vector<BlockMap> rowmaps(nrows);
  std::vector<int64_t> rowpairs(nrows, 0);
  for (auto& bm : rowmaps) bm.k = k;
  const bool dense = V.ig->level == 1;
  auto work_rows = [&](int tid) {
    PixelWalk Wk;
    Suffix Sx;
    Rows R;
    for (int tr = tid; tr < nrows; tr += threads) {
      BlockMap& bm = rowmaps[tr];
      for (int tx = 0; tx < V.L.tw; ++tx) {
        const int t = tr * V.L.tw + tx;
        const int* order = (const int*)&V.L.gids[V.L.start[t]];
        const size_t len = V.L.end[t] - V.L.start[t];
        for (int py = tr * tile; py < std::min(H, (tr + 1) * tile); ++py)
          for (int px = tx * tile; px < std::min(W, (tx + 1) * tile); ++px) {
            const double x = px + 0.5, y = py + 0.5;
            walk_pixel(order, len, x, y, V.pr, *V.gt, *V.rp, Wk);
            rowpairs[tr] += (int64_t)Wk.c.size();
            pixel_suffix(Wk, F, Sx);
            for (int ci = 0; ci < (int)Wk.c.size(); ++ci) {
              const int g = Wk.c[ci].gid;
              pixel_rows(Wk, Sx, ci, x, y, F, dp, dp_index, *V.ig, dense, R);
              accumulate_rows(R, &V.gt->p[(size_t)g * k], V.ig->level, bm.get(g));
            }
          }
      }
    }
  };
  {
    std::vector<std::thread> th;
    for (int t = 0; t < threads; ++t) th.emplace_back(work_rows, t);
    for (auto& x : th) x.join();
  }
  // merge rows in order
  std::map<int, Blocks> merged;
  BlocksResult out;
  out.k = k;
  for (int tr = 0; tr < nrows; ++tr) {
    out.pairs += rowpairs[tr];
    for (int g : rowmaps[tr].order) {
      Blocks& src = rowmaps[tr].m[g];
      auto it = merged.find(g);
      if (it == merged.end()) {
        merged.emplace(g, std::move(src));
      } else {
        for (size_t i = 0; i < src.rgb.size(); ++i) it->second.rgb[i] += src.rgb[i];
        for (size_t i = 0; i < src.d.size(); ++i) it->second.d[i] += src.d[i];
        for (size_t i = 0; i < src.o.size(); ++i) it->second.o[i] += src.o[i];
        it->second.a2 += src.a2;
      }
    }
    rowmaps[tr].m.clear();
  }
  for (auto& kv : merged) {
    if (!dense) finish_level2(kv.second, &V.gt->p[(size_t)kv.first * k], k);
    out.gids.push_back(kv.first);
    out.blocks.push_back(std::move(kv.second));
  }
  return out;
}

// Textbook Cholesky log-determinant; NaN if the matrix is not positive definite.
double chol_logdet(const double* A, int l) {
  std::vector<double> L((size_t)l * l, 0.0);
  double ld = 0.0;
  for (int j = 0; j < l; ++j) {
    double d = A[(size_t)j * l + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * l + k] * L[(size_t)j * l + k];
    if (!(d > 0.0)) return NAN;
    const double ljj = std::sqrt(d);
    L[(size_t)j * l + j] = ljj;
    ld += 2.0 * std::log(ljj);
    for (int i = j + 1; i < l; ++i) {
      double v = A[(size_t)i * l + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * l + k] * L[(size_t)j * l + k];
      L[(size_t)i * l + j] = v / ljj;
    }
  }
  return ld;
}

// trace(A^-1) of an SPD l x l matrix: A = L L^T, A^-1 = L^-T L^-1, so the trace is the sum
// of the squared entries of L^-1 (textbook Cholesky and forward substitution, column by column).
double chol_trace_inv(const double* A, int l) {
  std::vector<double> L((size_t)l * l, 0.0);
  for (int j = 0; j < l; ++j) {
    double d = A[(size_t)j * l + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * l + k] * L[(size_t)j * l + k];
    if (!(d > 0.0)) return NAN;
    const double ljj = std::sqrt(d);
    L[(size_t)j * l + j] = ljj;
    for (int i = j + 1; i < l; ++i) {
      double v = A[(size_t)i * l + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * l + k] * L[(size_t)j * l + k];
      L[(size_t)i * l + j] = v / ljj;
    }
  }
  double tr = 0.0;
  std::vector<double> x(l);
  for (int c = 0; c < l; ++c) {  // column c of L^-1: solve L x = e_c
    for (int i = 0; i < l; ++i) {
      double v = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) v -= L[(size_t)i * l + k] * x[k];
      x[i] = v / L[(size_t)i * l + i];
      tr += x[i] * x[i];
    }
  }
  return tr;
}

inline int block_len(int f, int k) { return f == 0 ? 14 : (f == 1 ? NGEO : NGEO + k); }
inline const std::vector<double>& block_of(const Blocks& b, int f) { return f == 0 ? b.rgb : (f == 1 ? b.d : b.o); }
inline std::vector<double>& block_of(Blocks& b, int f) { return f == 0 ? b.rgb : (f == 1 ? b.d : b.o); }

// IG_f(T, c) = sum_g [logdet(H_T,g + c_g A_c,g) - logdet(H_T,g)] (Eqs. 5, 6, 9). With the
// trace criterion the per-Gaussian term is the reduction of the covariance trace,
// trace(H_T,g^-1) - trace((H_T,g + c_g A_c,g)^-1), and out[] holds its sum R_f.
void info_gain(const BlocksResult& cand, const std::map<int, Blocks>& HT, const GaussTerms& gt,
               const or_ig& ig, int k, double out[3], std::vector<std::array<double, 3>>* per_g) {
  out[0] = out[1] = out[2] = 0.0;
  if (per_g) per_g->assign(cand.gids.size(), {0.0, 0.0, 0.0});
  for (size_t i = 0; i < cand.gids.size(); ++i) {
    const int g = cand.gids[i];
    const double cg = gt.conf[g];
    if (cg == 0.0) continue;
    auto it = HT.find(g);
    for (int f = 0; f < 3; ++f) {
      if (!((ig.outputs >> f) & 1)) continue;
      const int l = block_len(f, k);
      std::vector<double> Hm((size_t)l * l, 0.0), M((size_t)l * l, 0.0);
      if (it != HT.end()) {
        Hm = block_of(it->second, f);
      } else {
        for (int d = 0; d < l; ++d) Hm[(size_t)d * l + d] = ig.lambda_prior;
      }
      const std::vector<double>& A = block_of(cand.blocks[i], f);
      for (size_t e = 0; e < M.size(); ++e) M[e] = Hm[e] + cg * A[e];
      const double d = ig.criterion == 1 ? chol_trace_inv(Hm.data(), l) - chol_trace_inv(M.data(), l)
                                         : chol_logdet(M.data(), l) - chol_logdet(Hm.data(), l);
      out[f] += d;
      if (per_g) (*per_g)[i][f] = d;
    }
  }
}

std::map<int, Blocks> build_train(const std::vector<BlocksResult>& tv, const GaussTerms& gt,
                                  const or_ig& ig, int k) {
  std::map<int, Blocks> HT;
  for (const auto& br : tv)
    for (size_t i = 0; i < br.gids.size(); ++i) {
      const int g = br.gids[i];
      auto it = HT.find(g);
      if (it == HT.end()) {
        Blocks b;
        for (int f = 0; f < 3; ++f) {
          const int l = block_len(f, k);
          auto& v = block_of(b, f);
          v.assign((size_t)l * l, 0.0);
          for (int d = 0; d < l; ++d) v[(size_t)d * l + d] = ig.lambda_prior;
        }
        it = HT.emplace(g, std::move(b)).first;
      }
      const double w = ig.conf_on_train ? gt.conf[g] : 1.0;
      for (int f = 0; f < 3; ++f) {
        auto& dst = block_of(it->second, f);
        const auto& src = block_of(br.blocks[i], f);
        for (size_t e = 0; e < dst.size(); ++e) dst[e] += w * src[e];
      }
    }
  return HT;
}

}  // namespace

// ========================================================================================
// C API (called from the tests through ctypes)
// ========================================================================================
extern "C" {

int or_version() { return 1; }

int or_gaussian_terms(const or_scene* s, const or_ig* ig, double* p, double* kappa, double* sigma,
                      double* conf, int32_t* amax) {
  GaussTerms gt = gaussian_terms(*s, *ig);
  std::memcpy(p, gt.p.data(), gt.p.size() * sizeof(double));
  std::memcpy(kappa, gt.kappa.data(), gt.kappa.size() * sizeof(double));
  std::memcpy(sigma, gt.sigma.data(), gt.sigma.size() * sizeof(double));
  std::memcpy(conf, gt.conf.data(), gt.conf.size() * sizeof(double));
  std::memcpy(amax, gt.amax.data(), gt.amax.size() * sizeof(int32_t));
  return 0;
}

// Per-Gaussian projection. Outputs are [n] or [c][n] arrays; rect is [4][n] (x0, y0, x1, y1).
int or_project(const or_scene* s, const or_camera* cam, const or_raster* rp, double* z, uint32_t* zkey,
               double* m2, double* cov, double* conic, int32_t* radius, int32_t* rect, uint8_t* valid) {
  const int n = s->n;
  for (int g = 0; g < n; ++g) {
    Proj P = project_one(*s, g, *cam, *rp);
    z[g] = P.z;
    zkey[g] = P.valid ? P.zkey : 0xFFFFFFFFu;
    m2[g] = P.mx; m2[n + g] = P.my;
    for (int i = 0; i < 3; ++i) { cov[(size_t)i * n + g] = P.cov[i]; conic[(size_t)i * n + g] = P.conic[i]; }
    radius[g] = P.valid ? P.radius : 0;
    for (int i = 0; i < 4; ++i) rect[(size_t)i * n + g] = P.valid ? P.rect[i] : 0;
    valid[g] = P.valid ? 1 : 0;
  }
  return 0;
}

// Sorted tile lists. Returns M; writes keys/gids only when cap >= M. ranges: [2][tiles].
int64_t or_lists(const or_scene* s, const or_camera* cam, const or_raster* rp, int64_t cap,
                 uint64_t* keys, uint32_t* gids, uint32_t* ranges) {
  const int n = s->n;
  std::vector<Proj> pr(n);
  for (int g = 0; g < n; ++g) pr[g] = project_one(*s, g, *cam, *rp);
  Lists L = build_lists(pr, cam->width, cam->height, rp->tile);
  const int64_t M = (int64_t)L.gids.size();
  if (cap >= M && keys && gids && ranges) {  // a call with no outputs only asks for M
    std::memcpy(keys, L.keys.data(), M * sizeof(uint64_t));
    std::memcpy(gids, L.gids.data(), M * sizeof(uint32_t));
    const int nt = L.tw * L.th;
    for (int t = 0; t < nt; ++t) { ranges[t] = L.start[t]; ranges[nt + t] = L.end[t]; }
  }
  return M;
}

// Rendered images, [c][H][W] planes. brute != 0 composites every in-front Gaussian in
// (f32 depth, gid) order at every pixel, without tiles. Any output pointer may be NULL.
int or_render(const or_scene* s, const or_camera* cam, const or_raster* rp, const or_ig* ig, int brute,
              int threads, double* rgb, double* depth, double* obj, double* objp, double* tfin,
              int32_t* id, double* kbar, int32_t* ncontrib, uint8_t* ambiguous) {
  GaussTerms gt = gaussian_terms(*s, *ig);
  ViewCtx V{s, cam, rp, ig, &gt};
  view_setup(V);
  if (brute) build_brute(V);
  const int n = s->n, k = s->k, W = cam->width, H = cam->height;
  const size_t HW = (size_t)W * H;
  auto work = [&](int tid, int nth) {
    PixelWalk Wk;
    for (int py = tid; py < H; py += nth)
      for (int px = 0; px < W; ++px) {
        const int* order;
        size_t len;
        if (brute) {
          order = V.brute.data();
          len = V.brute.size();
        } else {
          const int t = (py / rp->tile) * V.L.tw + px / rp->tile;
          order = (const int*)&V.L.gids[V.L.start[t]];
          len = V.L.end[t] - V.L.start[t];
        }
        walk_pixel(order, len, px + 0.5, py + 0.5, V.pr, gt, *rp, Wk);
        double C[3] = {0, 0, 0}, D = 0, kb = 0;
        std::vector<double> Op(k, 0.0);
        for (const Contrib& c : Wk.c) {
          for (int ch = 0; ch < 3; ++ch) C[ch] += s->rgb[(size_t)ch * n + c.gid] * c.a;
          D += V.pr[c.gid].z * c.a;
          for (int m = 0; m < k; ++m) Op[m] += gt.p[(size_t)c.gid * k + m] * c.a;
          kb += gt.kappa[c.gid] * c.a;
        }
        const size_t pix = (size_t)py * W + px;
        double sumo = 0.0;
        for (int m = 0; m < k; ++m) sumo += Op[m];
        std::vector<double> O = Op;
        O[0] += 1.0 - sumo;  // Eq. 2: residual to the background channel
        int am = 0;
        for (int m = 1; m < k; ++m)
          if (O[m] > O[am]) am = m;
        if (rgb) for (int ch = 0; ch < 3; ++ch) rgb[ch * HW + pix] = C[ch];
        if (depth) depth[pix] = D;
        if (obj) for (int m = 0; m < k; ++m) obj[m * HW + pix] = O[m];
        if (objp) for (int m = 0; m < k; ++m) objp[m * HW + pix] = Op[m];
        if (tfin) tfin[pix] = Wk.t_final;
        if (id) id[pix] = am;
        if (kbar) kbar[pix] = Wk.c.empty() ? 0.0 : kb / (1.0 - Wk.t_final);
        if (ncontrib) ncontrib[pix] = (int32_t)Wk.c.size();
        if (ambiguous) ambiguous[pix] = Wk.ambiguous ? 1 : 0;
      }
  };
  threads = std::max(1, threads);
  std::vector<std::thread> th;
  for (int t = 0; t < threads; ++t) th.emplace_back(work, t, threads);
  for (auto& x : th) x.join();
  return 0;
}

// Per-view information blocks (unweighted A^f_g) of every touched Gaussian.
// Gradient of a scalar loss through the rendered images (refinement step, Sec. III-A.2,
// with the compositing of Eq. 1-2): for every Gaussian, grad = sum over pixels and channels
// of (dL / d out) times the row d out / d theta, theta = (mu 3, log-scale 3, raw quaternion
// 4, opacity logit 1 | rgb 3 | object logits k). The rows are the ones the information blocks
// are built from; the object rows enter through d O_m / d alpha and the softmax Jacobian.
// g_rgb [3][H][W], g_depth [H][W], g_obj [k][H][W] (gradient w.r.t. O of Eq. 2 when
// obj_eq2, else O'); any may be NULL. grad [n][14 + k] is overwritten.
int or_render_grad(const or_scene* s, const or_camera* cam, const or_raster* rp, const or_ig* ig, int threads,
                   const double* g_rgb, const double* g_depth, const double* g_obj, double* grad) {
  GaussTerms gt = gaussian_terms(*s, *ig);
  ViewCtx V{s, cam, rp, ig, &gt};
  view_setup(V);
  const int n = s->n, k = s->k, W = cam->width, H = cam->height, tile = rp->tile;
  const size_t HW = (size_t)W * H;
  const int L = NGEO + 3 + k;
  std::vector<int> dp_index(n, -1), valid_ids;
  for (int g = 0; g < n; ++g)
    if (V.pr[g].valid) { dp_index[g] = (int)valid_ids.size(); valid_ids.push_back(g); }
  std::vector<DualProj> dp(valid_ids.size());
  for (size_t i = 0; i < valid_ids.size(); ++i) dp[i] = project_dual(*s, valid_ids[i], *cam, *rp);
  Features F{s, &V.pr, &gt};
  const int nrows = V.L.th;
  std::vector<std::map<int, std::vector<double>>> rowacc(nrows);
  auto work = [&](int tid, int nth) {
    PixelWalk Wk;
    Suffix Sx;
    Rows R;
    std::vector<double> go(k);
    for (int tr = tid; tr < nrows; tr += nth) {
      auto& acc = rowacc[tr];
      for (int tx = 0; tx < V.L.tw; ++tx) {
        const int t = tr * V.L.tw + tx;
        const int* order = (const int*)&V.L.gids[V.L.start[t]];
        const size_t len = V.L.end[t] - V.L.start[t];
        for (int py = tr * tile; py < std::min(H, (tr + 1) * tile); ++py)
          for (int px = tx * tile; px < std::min(W, (tx + 1) * tile); ++px) {
            const double x = px + 0.5, y = py + 0.5;
            const size_t pix = (size_t)py * W + px;
            walk_pixel(order, len, x, y, V.pr, gt, *rp, Wk);
            if (Wk.c.empty()) continue;
            pixel_suffix(Wk, F, Sx);
            double gc[3];
            for (int ch = 0; ch < 3; ++ch) gc[ch] = g_rgb ? g_rgb[ch * HW + pix] : 0.0;
            const double gd = g_depth ? g_depth[pix] : 0.0;
            for (int m = 0; m < k; ++m) go[m] = g_obj ? g_obj[m * HW + pix] : 0.0;
            for (int ci = 0; ci < (int)Wk.c.size(); ++ci) {
              const int g = Wk.c[ci].gid;
              pixel_rows(Wk, Sx, ci, x, y, F, dp, dp_index, *ig, false, R);
              std::vector<double>& v = acc[g];
              if (v.empty()) v.assign(L, 0.0);
              double wo_dot = 0.0;
              for (int m = 0; m < k; ++m) wo_dot += go[m] * R.wo[m];
              for (int i = 0; i < NGEO; ++i) {
                double a = gd * R.d[i] + wo_dot * R.gvec[i];
                for (int ch = 0; ch < 3; ++ch) a += gc[ch] * R.rgb[ch][i];
                v[i] += a;
              }
              for (int ch = 0; ch < 3; ++ch) v[NGEO + ch] += gc[ch] * R.rgb[ch][NGEO + ch];
              const double* pg = &gt.p[(size_t)g * k];
              double dot = 0.0;
              for (int m = 0; m < k; ++m) dot += go[m] * pg[m];
              for (int j = 0; j < k; ++j) v[NGEO + 3 + j] += R.a * pg[j] * (go[j] - dot);
            }
          }
      }
    }
  };
  threads = std::max(1, threads);
  {
    std::vector<std::thread> th;
    for (int t = 0; t < threads; ++t) th.emplace_back(work, t, threads);
    for (auto& x : th) x.join();
  }
  std::fill(grad, grad + (size_t)n * L, 0.0);
  for (int tr = 0; tr < nrows; ++tr)
    for (auto& kv : rowacc[tr])
      for (int i = 0; i < L; ++i) grad[(size_t)kv.first * L + i] += kv.second[i];
  return 0;
}

void* or_view_blocks(const or_scene* s, const or_camera* cam, const or_raster* rp, const or_ig* ig, int threads) {
  GaussTerms gt = gaussian_terms(*s, *ig);
  ViewCtx V{s, cam, rp, ig, &gt};
  view_setup(V);
  return new BlocksResult(view_blocks(V, threads));
}
int64_t or_blocks_count(void* h) { return (int64_t)static_cast<BlocksResult*>(h)->gids.size(); }
int64_t or_blocks_pairs(void* h) { return static_cast<BlocksResult*>(h)->pairs; }
int or_blocks_get(void* h, int64_t i, int32_t* gid, double* a_rgb, double* a_d, double* a_o) {
  auto* b = static_cast<BlocksResult*>(h);
  *gid = b->gids[i];
  if (a_rgb) std::memcpy(a_rgb, b->blocks[i].rgb.data(), b->blocks[i].rgb.size() * sizeof(double));
  if (a_d) std::memcpy(a_d, b->blocks[i].d.data(), b->blocks[i].d.size() * sizeof(double));
  if (a_o) std::memcpy(a_o, b->blocks[i].o.data(), b->blocks[i].o.size() * sizeof(double));
  return 0;
}
void or_blocks_free(void* h) { delete static_cast<BlocksResult*>(h); }

double or_logdet(int l, const double* A) { return chol_logdet(A, l); }
double or_trace_inv(int l, const double* A) { return chol_trace_inv(A, l); }

// Jacobian rows at pixel (px, py) for every contributor, front to back. Returns the number
// of contributors (rows written only when it is <= cap): contrib [cap] gids, rows_rgb
// [cap][3][14], rows_d [cap][11], rows_o [cap][k][11+k].
int or_pixel_rows(const or_scene* s, const or_camera* cam, const or_raster* rp, const or_ig* ig,
                  int px, int py, int cap, int32_t* contrib, double* rows_rgb, double* rows_d, double* rows_o) {
  GaussTerms gt = gaussian_terms(*s, *ig);
  ViewCtx V{s, cam, rp, ig, &gt};
  view_setup(V);
  const int t = (py / rp->tile) * V.L.tw + px / rp->tile;
  PixelWalk Wk;
  walk_pixel((const int*)&V.L.gids[V.L.start[t]], V.L.end[t] - V.L.start[t], px + 0.5, py + 0.5, V.pr, gt, *rp, Wk);
  const int nc = (int)Wk.c.size();
  if (nc > cap) return nc;
  std::vector<int> dp_index(s->n, -1);
  std::vector<DualProj> dp;
  for (const Contrib& c : Wk.c) { dp_index[c.gid] = (int)dp.size(); dp.push_back(project_dual(*s, c.gid, *cam, *rp)); }
  Features F{s, &V.pr, &gt};
  Suffix Sx;
  pixel_suffix(Wk, F, Sx);
  Rows R;
  const int k = s->k, lo = NGEO + k;
  for (int ci = 0; ci < nc; ++ci) {
    pixel_rows(Wk, Sx, ci, px + 0.5, py + 0.5, F, dp, dp_index, *ig, true, R);
    contrib[ci] = Wk.c[ci].gid;
    for (int ch = 0; ch < 3; ++ch) std::memcpy(&rows_rgb[((size_t)ci * 3 + ch) * 14], R.rgb[ch], 14 * sizeof(double));
    std::memcpy(&rows_d[(size_t)ci * NGEO], R.d, NGEO * sizeof(double));
    std::memcpy(&rows_o[(size_t)ci * k * lo], R.o.data(), (size_t)k * lo * sizeof(double));
  }
  return nc;
}

// Composites a fixed front-to-back sequence at (px, py): no cut, skip or stop decision,
// only the alpha clamp. out = [rgb 3, depth 1, object k (O or O' per ig->obj_eq2)].
// Used by finite-difference checks with the contributing set frozen.
int or_pixel_eval_frozen(const or_scene* s, const or_camera* cam, const or_raster* rp, const or_ig* ig,
                         int px, int py, int nseq, const int32_t* seq, double* out) {
  GaussTerms gt = gaussian_terms(*s, *ig);
  const int n = s->n, k = s->k;
  double T = 1.0;
  for (int i = 0; i < 4 + k; ++i) out[i] = 0.0;
  for (int i = 0; i < nseq; ++i) {
    const int g = seq[i];
    Proj P = project_one(*s, g, *cam, *rp);
    const double dx = px + 0.5 - P.mx, dy = py + 0.5 - P.my;
    const double q = P.conic[0] * dx * dx + 2.0 * P.conic[1] * dx * dy + P.conic[2] * dy * dy;
    const double alpha = std::min(rp->alpha_max, gt.sigma[g] * std::exp(-0.5 * q));
    const double a = alpha * T;
    for (int ch = 0; ch < 3; ++ch) out[ch] += s->rgb[(size_t)ch * n + g] * a;
    out[3] += P.z * a;
    for (int m = 0; m < k; ++m) out[4 + m] += gt.p[(size_t)g * k + m] * a;
    T *= 1.0 - alpha;
  }
  if (ig->obj_eq2) {
    double so = 0.0;
    for (int m = 0; m < k; ++m) so += out[4 + m];
    out[4] += 1.0 - so;
  }
  return 0;
}

// Full scoring: training information, normalisers (Eq. 10), candidate scores (Eq. 11),
// argmax (Eq. 5). ig_train [nt][3], ig_cand [nc][3], norm [3], scores [nc][4]
// (normalised rgb, depth, object, combined). Returns 0, or -5 when an enabled
// normaliser is not positive (scores then hold the raw gains only).
// Wall-clock seconds of the last or_score call: [0] training information and normalisers,
// [1] the candidates, then one entry per candidate (read by or_last_score_seconds; timing
// only, no arithmetic). or_set_setup_threads(t > 0) runs the training views of later calls on
// t threads instead of the call's own count (so that a single-threaded candidate timing does
// not wait for a single-threaded training set).
static std::vector<double> g_score_seconds(2, 0.0);
static int g_setup_threads = 0;

int or_last_score_seconds(double* out, int cap) {
  const int n = (int)g_score_seconds.size();
  for (int i = 0; i < n && i < cap; ++i) out[i] = g_score_seconds[i];
  return n;
}

void or_set_setup_threads(int t) { g_setup_threads = t; }

int or_score(const or_scene* s, int nt, const or_camera* train, int nc, const or_camera* cand,
             const or_raster* rp, const or_ig* ig, int threads, double* ig_train, double* ig_cand,
             double* norm, double* scores, int32_t* best, int64_t* stats /*[nc][2]: U, pairs*/,
             double* trace_total /*[3] S_T of the trace criterion, may be NULL*/) {
  using clock = std::chrono::steady_clock;
  const auto t_start = clock::now();
  g_score_seconds.assign(2 + (size_t)std::max(nc, 0), 0.0);
  GaussTerms gt = gaussian_terms(*s, *ig);
  const int k = s->k;
  std::vector<BlocksResult> tv;
  for (int t = 0; t < nt; ++t) {
    ViewCtx V{s, &train[t], rp, ig, &gt};
    view_setup(V);
    tv.push_back(view_blocks(V, g_setup_threads > 0 ? g_setup_threads : threads));
  }
  std::map<int, Blocks> HT = build_train(tv, gt, *ig, k);
  // trace criterion: f(V) = 1 / S_V with S_V = sum over all n Gaussians of trace(H_V,g^-1)
  // (block diagonal H; a Gaussian no training view touched has H_T,g = lambda I), so
  // f(T + c) - f(T) = 1 / (S_T - R) - 1 / S_T = R / (S_T (S_T - R)) for the reduction R.
  double st[3] = {0, 0, 0};
  if (ig->criterion == 1)
    for (int f = 0; f < 3; ++f) {
      const int l = block_len(f, k);
      for (const auto& kv : HT) st[f] += chol_trace_inv(block_of(kv.second, f).data(), l);
      st[f] += (double)(s->n - (int64_t)HT.size()) * l / ig->lambda_prior;
    }
  auto gain = [&](int f, double r) { return ig->criterion == 1 ? r / (st[f] * (st[f] - r)) : r; };
  double nf[3] = {0, 0, 0};
  for (int t = 0; t < nt; ++t) {
    double o[3];
    info_gain(tv[t], HT, gt, *ig, k, o, nullptr);
    for (int f = 0; f < 3; ++f) { ig_train[3 * t + f] = o[f]; nf[f] += gain(f, o[f]) / nt; }
  }
  if (trace_total)
    for (int f = 0; f < 3; ++f) trace_total[f] = st[f];
  tv.clear();
  for (int f = 0; f < 3; ++f) norm[f] = nf[f];
  int status = 0;
  for (int f = 0; f < 3; ++f)
    if (((ig->outputs >> f) & 1) && !(nf[f] > 0.0)) status = -5;
  const double beta[3] = {1.0, ig->beta_d, ig->beta_o};
  int b = -1;
  double bestv = -INFINITY;
  const auto t_cand = clock::now();
  for (int c = 0; c < nc; ++c) {
    const auto t_c = clock::now();
    ViewCtx V{s, &cand[c], rp, ig, &gt};
    view_setup(V);
    BlocksResult br = view_blocks(V, threads);
    double o[3];
    info_gain(br, HT, gt, *ig, k, o, nullptr);
    if (stats) { stats[2 * c] = (int64_t)br.gids.size(); stats[2 * c + 1] = br.pairs; }
    double tot = 0.0;
    for (int f = 0; f < 3; ++f) {
      ig_cand[3 * c + f] = o[f];
      const double v = (status == 0 && ((ig->outputs >> f) & 1)) ? gain(f, o[f]) / nf[f] : 0.0;
      scores[4 * c + f] = v;
      tot += beta[f] * v;
    }
    scores[4 * c + 3] = tot;
    if (status == 0 && tot > bestv) { bestv = tot; b = c; }
    g_score_seconds[2 + c] = std::chrono::duration<double>(clock::now() - t_c).count();
  }
  *best = b;
  g_score_seconds[0] = std::chrono::duration<double>(t_cand - t_start).count();
  g_score_seconds[1] = std::chrono::duration<double>(clock::now() - t_cand).count();
  return status;
}

// Training information blocks for inspection: fills H (weighted, with prior) for the
// requested Gaussians; returns the number of those touched by a training view.
int or_train_blocks(const or_scene* s, int nt, const or_camera* train, const or_raster* rp, const or_ig* ig,
                    int threads, int nq, const int32_t* query, double* h_rgb, double* h_d, double* h_o,
                    uint8_t* touched) {
  GaussTerms gt = gaussian_terms(*s, *ig);
  const int k = s->k, lo = NGEO + k;
  std::vector<BlocksResult> tv;
  for (int t = 0; t < nt; ++t) {
    ViewCtx V{s, &train[t], rp, ig, &gt};
    view_setup(V);
    tv.push_back(view_blocks(V, threads));
  }
  std::map<int, Blocks> HT = build_train(tv, gt, *ig, k);
  int cnt = 0;
  for (int i = 0; i < nq; ++i) {
    auto it = HT.find(query[i]);
    touched[i] = it != HT.end();
    cnt += touched[i];
    for (int f = 0; f < 3; ++f) {
      const int l = block_len(f, k);
      double* dst = f == 0 ? &h_rgb[(size_t)i * 196] : (f == 1 ? &h_d[(size_t)i * 121] : &h_o[(size_t)i * lo * lo]);
      if (it != HT.end()) {
        std::memcpy(dst, block_of(it->second, f).data(), (size_t)l * l * sizeof(double));
      } else {
        for (int e = 0; e < l * l; ++e) dst[e] = 0.0;
        for (int d = 0; d < l; ++d) dst[(size_t)d * l + d] = ig->lambda_prior;
      }
    }
  }
  return cnt;
}

}  // extern "C"
