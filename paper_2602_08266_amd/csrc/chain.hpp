// chain.hpp -- FP64 derivatives of one Gaussian's screen-space quantities w.r.t. its raw
// parameters, shared by the information-gain finalize and the backward rasterizer.
#pragma once

#include "common.hpp"

namespace ngs {

// dQ = -Q dSigma Q for the conic Q = (q00, q01, q11) and dSigma = [[da, db], [db, dc]].
__device__ inline void dconic(double q00, double q01, double q11, double da, double db, double dc, double* out) {
  out[0] = -(q00 * q00 * da + 2.0 * q00 * q01 * db + q01 * q01 * dc);
  out[1] = -(q00 * q01 * da + (q00 * q11 + q01 * q01) * db + q01 * q11 * dc);
  out[2] = -(q01 * q01 * da + 2.0 * q01 * q11 * db + q11 * q11 * dc);
}

// Hand chain rule of the projection (3DGS EWA splatting) in FP64: rows of P for
// (m_x, m_y, Q_xx, Q_xy, Q_yy, l) and the depth row, w.r.t. the 11 geometric parameters.
__device__ inline void chain_rule(const float* mean, const float* log_scale, const float* rot, int n, int g,
                           const DevCam& cam, double eps2d, double P[7][kNGeo]) {
  double W[9];
  for (int i = 0; i < 9; ++i) W[i] = cam.R[i];
  const double mu[3] = {mean[g], mean[n + g], mean[2 * n + g]};
  double X[3];
  for (int i = 0; i < 3; ++i) X[i] = W[3 * i] * mu[0] + W[3 * i + 1] * mu[1] + W[3 * i + 2] * mu[2] + cam.t[i];
  const double Z = X[2], fx = cam.fx, fy = cam.fy;
  const double iz = 1.0 / Z, iz2 = iz * iz, iz3 = iz2 * iz;
  const double Jp[6] = {fx * iz, 0.0, -fx * X[0] * iz2, 0.0, fy * iz, -fy * X[1] * iz2};
  double T[6];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) T[3 * i + j] = Jp[3 * i] * W[j] + Jp[3 * i + 1] * W[3 + j] + Jp[3 * i + 2] * W[6 + j];
  double s2[3];
  for (int i = 0; i < 3; ++i) { const double s = exp((double)log_scale[(size_t)i * n + g]); s2[i] = s * s; }
  const double q4[4] = {rot[g], rot[n + g], rot[2 * n + g], rot[3 * n + g]};
  const double qn = sqrt(q4[0] * q4[0] + q4[1] * q4[1] + q4[2] * q4[2] + q4[3] * q4[3]);
  const double w = q4[0] / qn, x = q4[1] / qn, y = q4[2] / qn, z = q4[3] / qn;
  const double Rg[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                        2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                        2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
  double S3[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) S3[3 * i + j] = Rg[3 * i] * s2[0] * Rg[3 * j] + Rg[3 * i + 1] * s2[1] * Rg[3 * j + 1] +
                                                Rg[3 * i + 2] * s2[2] * Rg[3 * j + 2];
  // V = Sigma3 T^T (3 x 2), Sigma2 = T V + eps I
  double V[6];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 2; ++j) V[2 * i + j] = S3[3 * i] * T[3 * j] + S3[3 * i + 1] * T[3 * j + 1] + S3[3 * i + 2] * T[3 * j + 2];
  const double a = T[0] * V[0] + T[1] * V[2] + T[2] * V[4] + eps2d;
  const double b = T[0] * V[1] + T[1] * V[3] + T[2] * V[5];
  const double c = T[3] * V[1] + T[4] * V[3] + T[5] * V[5] + eps2d;
  const double det = a * c - b * b;
  const double q00 = c / det, q01 = -b / det, q11 = a / det;
  for (int r = 0; r < 7; ++r)
    for (int j = 0; j < kNGeo; ++j) P[r][j] = 0.0;
  // mean: m through T, Q through the perspective Jacobian's dependence on X = W mu + t
  double dS[3][3];  // dSigma2 / dX_m as (da, db, dc)
  for (int m = 0; m < 3; ++m) {
    double dJ[6] = {0, 0, 0, 0, 0, 0};
    if (m == 0) dJ[2] = -fx * iz2;
    if (m == 1) dJ[5] = -fy * iz2;
    if (m == 2) { dJ[0] = -fx * iz2; dJ[2] = 2.0 * fx * X[0] * iz3; dJ[4] = -fy * iz2; dJ[5] = 2.0 * fy * X[1] * iz3; }
    double dT[6];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 3; ++j) dT[3 * i + j] = dJ[3 * i] * W[j] + dJ[3 * i + 1] * W[3 + j] + dJ[3 * i + 2] * W[6 + j];
    double B[4];
    for (int i = 0; i < 2; ++i)
      for (int j = 0; j < 2; ++j) B[2 * i + j] = dT[3 * i] * V[j] + dT[3 * i + 1] * V[2 + j] + dT[3 * i + 2] * V[4 + j];
    dS[m][0] = 2.0 * B[0];
    dS[m][1] = B[1] + B[2];
    dS[m][2] = 2.0 * B[3];
  }
  for (int j = 0; j < 3; ++j) {
    P[0][j] = T[j];
    P[1][j] = T[3 + j];
    double da = 0, db = 0, dc = 0;
    for (int m = 0; m < 3; ++m) { da += W[3 * m + j] * dS[m][0]; db += W[3 * m + j] * dS[m][1]; dc += W[3 * m + j] * dS[m][2]; }
    double o[3];
    dconic(q00, q01, q11, da, db, dc, o);
    P[2][j] = o[0]; P[3][j] = o[1]; P[4][j] = o[2];
    P[6][j] = W[6 + j];
  }
  // log-scales: dSigma3 = 2 s_i^2 r_i r_i^T
  for (int i = 0; i < 3; ++i) {
    const double u0 = T[0] * Rg[i] + T[1] * Rg[3 + i] + T[2] * Rg[6 + i];
    const double u1 = T[3] * Rg[i] + T[4] * Rg[3 + i] + T[5] * Rg[6 + i];
    double o[3];
    dconic(q00, q01, q11, 2.0 * s2[i] * u0 * u0, 2.0 * s2[i] * u0 * u1, 2.0 * s2[i] * u1 * u1, o);
    P[2][3 + i] = o[0]; P[3][3 + i] = o[1]; P[4][3 + i] = o[2];
  }
  // quaternion: Rg(q / |q|)
  double U[6];  // T Rg
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 3; ++j) U[3 * i + j] = T[3 * i] * Rg[j] + T[3 * i + 1] * Rg[3 + j] + T[3 * i + 2] * Rg[6 + j];
  const double dR[4][9] = {
      {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0},
      {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x},
      {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y},
      {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0}};
  const double qh[4] = {w, x, y, z};
  for (int j = 0; j < 4; ++j) {
    double dRg[9];
    for (int e = 0; e < 9; ++e) {
      double v = 0.0;
      for (int l = 0; l < 4; ++l) v += dR[l][e] * (((l == j) ? 1.0 : 0.0) - qh[l] * qh[j]) / qn;
      dRg[e] = v;
    }
    double dU[6];
    for (int i = 0; i < 2; ++i)
      for (int e = 0; e < 3; ++e) dU[3 * i + e] = T[3 * i] * dRg[e] + T[3 * i + 1] * dRg[3 + e] + T[3 * i + 2] * dRg[6 + e];
    double B[4];
    for (int i = 0; i < 2; ++i)
      for (int k2 = 0; k2 < 2; ++k2)
        B[2 * i + k2] = dU[3 * i] * s2[0] * U[3 * k2] + dU[3 * i + 1] * s2[1] * U[3 * k2 + 1] + dU[3 * i + 2] * s2[2] * U[3 * k2 + 2];
    double o[3];
    dconic(q00, q01, q11, 2.0 * B[0], B[1] + B[2], 2.0 * B[3], o);
    P[2][6 + j] = o[0]; P[3][6 + j] = o[1]; P[4][6 + j] = o[2];
  }
  P[5][10] = 1.0;
}

}  // namespace ngs
