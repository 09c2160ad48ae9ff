// The camera model of the method on the device: projection Jacobians
// (Sec. 5.1), shared by the scene stage and the incremental update.
#pragma once

#include <hip/hip_runtime.h>

namespace ucov {

struct Jac {
  double jp[2][9];
  double jx[2][3];
  double x[3];
};

// u = f d pi + c0, pi = x[0:2]/x[2], x = R(r)(X - C), d = 1 + k1 rho2 + k2 rho2^2.
//   du/dpi  = f (d I + 2 (k1 + 2 k2 rho2) pi pi^T)
//   dpi/dx  = [[1, 0, -pi0], [0, 1, -pi1]] / x2
//   dx/dX   = R,  dx/dC = -R,  dx/dr = -[x]x J_l(r)
// with J_l(r) = I + (1 - cos t)/t^2 [r]x + (t - sin t)/t^3 [r]x^2 the left
// Jacobian of SO(3), and du/df = d pi, du/dk1 = f rho2 pi, du/dk2 = f rho2^2 pi.
__device__ inline void projection_jacobian(const double *cam, const double *X, Jac &J) {
  const double r0 = cam[0], r1 = cam[1], r2 = cam[2];
  const double t2 = r0 * r0 + r1 * r1 + r2 * r2;
  double a, b, c;  // sin t / t, (1 - cos t)/t^2, (t - sin t)/t^3
  if (t2 < 1e-4) {
    // Taylor series in t^2 (truncation below 1e-20 for t < 0.01)
    a = 1.0 + t2 * (-1.0 / 6 + t2 * (1.0 / 120 + t2 * (-1.0 / 5040 + t2 / 362880)));
    b = 0.5 + t2 * (-1.0 / 24 + t2 * (1.0 / 720 + t2 * (-1.0 / 40320 + t2 / 3628800)));
    c = 1.0 / 6 + t2 * (-1.0 / 120 + t2 * (1.0 / 5040 + t2 * (-1.0 / 362880 + t2 / 39916800)));
  } else {
    const double t = sqrt(t2);
    double s, co, sh, chh;
    sincos(t, &s, &co);
    sincos(0.5 * t, &sh, &chh);
    a = s / t;
    b = 2.0 * sh * sh / t2;  // (1 - cos t) / t^2 without cancellation
    c = (t - s) / (t2 * t);
  }
  // K = [r]x, R = I + a K + b K^2
  const double K[3][3] = {{0, -r2, r1}, {r2, 0, -r0}, {-r1, r0, 0}};
  double K2[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      K2[i][j] = K[i][0] * K[0][j] + K[i][1] * K[1][j] + K[i][2] * K[2][j];
  double R[3][3], Jl[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double id = (i == j) ? 1.0 : 0.0;
      R[i][j] = id + a * K[i][j] + b * K2[i][j];
      Jl[i][j] = id + b * K[i][j] + c * K2[i][j];
    }
  const double v0 = X[0] - cam[3], v1 = X[1] - cam[4], v2 = X[2] - cam[5];
  double x[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) x[i] = R[i][0] * v0 + R[i][1] * v1 + R[i][2] * v2;
  J.x[0] = x[0];
  J.x[1] = x[1];
  J.x[2] = x[2];
  const double iz = 1.0 / x[2];
  const double p0 = x[0] * iz, p1 = x[1] * iz;
  const double rho2 = p0 * p0 + p1 * p1;
  const double f = cam[6], k1 = cam[7], k2 = cam[8];
  const double d = 1.0 + k1 * rho2 + k2 * rho2 * rho2;
  const double e = 2.0 * (k1 + 2.0 * k2 * rho2);
  // du/dpi (symmetric 2x2)
  const double D00 = f * (d + e * p0 * p0), D01 = f * e * p0 * p1, D11 = f * (d + e * p1 * p1);
  // G = du/dx = du/dpi * dpi/dx (2x3)
  double G[2][3];
  G[0][0] = D00 * iz;
  G[0][1] = D01 * iz;
  G[0][2] = -(D00 * p0 + D01 * p1) * iz;
  G[1][0] = D01 * iz;
  G[1][1] = D11 * iz;
  G[1][2] = -(D01 * p0 + D11 * p1) * iz;
  // dx/dr = -[x]x Jl
  const double Xs[3][3] = {{0, -x[2], x[1]}, {x[2], 0, -x[0]}, {-x[1], x[0], 0}};
  double DR[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      DR[i][j] = -(Xs[i][0] * Jl[0][j] + Xs[i][1] * Jl[1][j] + Xs[i][2] * Jl[2][j]);
#pragma unroll
  for (int p = 0; p < 2; ++p) {
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double gr = G[p][0] * DR[0][j] + G[p][1] * DR[1][j] + G[p][2] * DR[2][j];
      const double gx = G[p][0] * R[0][j] + G[p][1] * R[1][j] + G[p][2] * R[2][j];
      J.jp[p][j] = gr;
      J.jp[p][3 + j] = -gx;
      J.jx[p][j] = gx;
    }
  }
  J.jp[0][6] = d * p0;
  J.jp[1][6] = d * p1;
  J.jp[0][7] = f * rho2 * p0;
  J.jp[1][7] = f * rho2 * p1;
  J.jp[0][8] = f * rho2 * rho2 * p0;
  J.jp[1][8] = f * rho2 * rho2 * p1;
}

__device__ inline bool finite9(const double *v, int k) {
  for (int i = 0; i < k; ++i)
    if (!isfinite(v[i])) return false;
  return true;
}

}  // namespace ucov
