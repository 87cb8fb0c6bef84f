// Pair basis on the device: Chebyshev radial functions x smooth cutoff x real
// spherical harmonics, and their gradients (paper, Section V.B: B2 descriptors from
// radial functions and spherical harmonics).
//
//   R_n(r)  = T_n(x) f_c(r),  x = 2r/r_c - 1,  f_c = (r_c - r)^2 for r < r_c
//   R_n'(r) = n U_{n-1}(x) (2/r_c) f_c - 2 T_n(x) (r_c - r)
//   Y_lm(u) = P_lm(u) for a unit vector u, with P_lm the degree-l homogeneous
//             (solid harmonic) polynomial normalised so that the Y_lm are orthonormal
//   grad_Delta Y_lm(Delta/r) = (grad P_lm(u) - l P_lm(u) u) / r   (Euler's identity
//             u . grad P = l P for a homogeneous polynomial)
#pragma once

#include "common.h"

namespace flare {

// normalisation constants of the real spherical harmonics, l <= 3
constexpr float kY0 = 0.28209479177387814f;    // 1/(2 sqrt(pi))
constexpr float kY1 = 0.48860251190291992f;    // sqrt(3/(4 pi))
constexpr float kY2a = 1.0925484305920792f;    // (1/2) sqrt(15/pi)
constexpr float kY20 = 0.31539156525252005f;   // (1/4) sqrt(5/pi)
constexpr float kY22 = 0.54627421529603959f;   // (1/4) sqrt(15/pi)
constexpr float kY33 = 0.59004358992664352f;   // (1/4) sqrt(35/(2 pi))
constexpr float kY32a = 2.8906114426405538f;   // (1/2) sqrt(105/pi)
constexpr float kY31 = 0.45704579946446572f;   // (1/4) sqrt(21/(2 pi))
constexpr float kY30 = 0.37317633259011540f;   // (1/4) sqrt(7/pi)
constexpr float kY32b = 1.4453057213202769f;   // (1/4) sqrt(105/pi)

__device__ __forceinline__ void sph_harm(float x, float y, float z, float* Y) {
  const float xx = x * x, yy = y * y, zz = z * z;
  Y[0] = kY0;
  Y[1] = kY1 * y;
  Y[2] = kY1 * z;
  Y[3] = kY1 * x;
  Y[4] = kY2a * x * y;
  Y[5] = kY2a * y * z;
  Y[6] = kY20 * (2.f * zz - xx - yy);
  Y[7] = kY2a * x * z;
  Y[8] = kY22 * (xx - yy);
  Y[9] = kY33 * y * (3.f * xx - yy);
  Y[10] = kY32a * x * y * z;
  Y[11] = kY31 * y * (4.f * zz - xx - yy);
  Y[12] = kY30 * z * (2.f * zz - 3.f * xx - 3.f * yy);
  Y[13] = kY31 * x * (4.f * zz - xx - yy);
  Y[14] = kY32b * z * (xx - yy);
  Y[15] = kY33 * x * (xx - 3.f * yy);
}

// g[lm][3] = grad of the homogeneous polynomial P_lm at (x, y, z)
__device__ __forceinline__ void sph_harm_poly_grad(float x, float y, float z, float (*g)[3]) {
  const float xx = x * x, yy = y * y, zz = z * z;
  g[0][0] = 0.f; g[0][1] = 0.f; g[0][2] = 0.f;
  g[1][0] = 0.f; g[1][1] = kY1; g[1][2] = 0.f;
  g[2][0] = 0.f; g[2][1] = 0.f; g[2][2] = kY1;
  g[3][0] = kY1; g[3][1] = 0.f; g[3][2] = 0.f;
  g[4][0] = kY2a * y; g[4][1] = kY2a * x; g[4][2] = 0.f;
  g[5][0] = 0.f; g[5][1] = kY2a * z; g[5][2] = kY2a * y;
  g[6][0] = -2.f * kY20 * x; g[6][1] = -2.f * kY20 * y; g[6][2] = 4.f * kY20 * z;
  g[7][0] = kY2a * z; g[7][1] = 0.f; g[7][2] = kY2a * x;
  g[8][0] = 2.f * kY22 * x; g[8][1] = -2.f * kY22 * y; g[8][2] = 0.f;
  g[9][0] = 6.f * kY33 * x * y; g[9][1] = 3.f * kY33 * (xx - yy); g[9][2] = 0.f;
  g[10][0] = kY32a * y * z; g[10][1] = kY32a * x * z; g[10][2] = kY32a * x * y;
  g[11][0] = -2.f * kY31 * x * y; g[11][1] = kY31 * (4.f * zz - xx - 3.f * yy); g[11][2] = 8.f * kY31 * y * z;
  g[12][0] = -6.f * kY30 * x * z; g[12][1] = -6.f * kY30 * y * z; g[12][2] = kY30 * (6.f * zz - 3.f * xx - 3.f * yy);
  g[13][0] = kY31 * (4.f * zz - 3.f * xx - yy); g[13][1] = -2.f * kY31 * x * y; g[13][2] = 8.f * kY31 * x * z;
  g[14][0] = 2.f * kY32b * x * z; g[14][1] = -2.f * kY32b * y * z; g[14][2] = kY32b * (xx - yy);
  g[15][0] = 3.f * kY33 * (xx - yy); g[15][1] = -6.f * kY33 * x * y; g[15][2] = 0.f;
}

__device__ __forceinline__ int lm_l(int lm) { return lm == 0 ? 0 : (lm < 4 ? 1 : (lm < 9 ? 2 : 3)); }

// R_n(r), n = 0..NR-1. x = r (2/r_c) - 1: the factor 2/r_c is loop-invariant for the
// callers, which evaluate it once.
__device__ __forceinline__ void radial(float r, float rc, float* R) {
  const float x = r * (2.f / rc) - 1.f;
  const float fc = (rc - r) * (rc - r);
  float t0 = 1.f, t1 = x;
  R[0] = fc;
  R[1] = x * fc;
#pragma unroll
  for (int n = 2; n < NR; ++n) {
    const float t2 = 2.f * x * t1 - t0;
    R[n] = t2 * fc;
    t0 = t1;
    t1 = t2;
  }
}

// R_n(r) and dR_n/dr = T_n'(x) (2/r_c) f_c + T_n(x) f_c', with T_n' = n U_{n-1}
__device__ __forceinline__ void radial_d(float r, float rc, float* R, float* dR) {
  const float dxdr = 2.f / rc;
  const float x = r * dxdr - 1.f;
  const float q = rc - r;
  const float fc = q * q;
  const float dfc = -2.f * q;
  const float cf = dxdr * fc;
  float T[NR], U[NR];
  T[0] = 1.f;
  T[1] = x;
  U[0] = 1.f;
  U[1] = 2.f * x;
#pragma unroll
  for (int n = 2; n < NR; ++n) {
    T[n] = 2.f * x * T[n - 1] - T[n - 2];
    U[n] = 2.f * x * U[n - 1] - U[n - 2];
  }
  R[0] = fc;
  dR[0] = dfc;
#pragma unroll
  for (int n = 1; n < NR; ++n) {
    R[n] = T[n] * fc;
    dR[n] = ((float)n * cf) * U[n - 1] + T[n] * dfc;
  }
}

}  // namespace flare
