// Device geometry and wave-level helpers shared by the window solver
// (kernels.hip) and the motion-only solver (pnp.hip).
//
// Residual and kernel (paper Sec. 2.2, Eq. 2): r = pi(T_cb T_bw p) - o with a
// pinhole pi, the Huber kernel on s = |r|^2; pose updates by the left
// perturbation T <- Exp(xi) T, xi = (rho, phi).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace ba {

// 1/x and 1/sqrt(x) in FP64: the hardware estimates refined by two Newton
// steps each (a few ulp for finite normal x; not correctly rounded).
__device__ __forceinline__ double recip_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double rsqrt_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  double h = fma(-x * r, r, 1.0);   // r <- r + r (1 - x r^2) / 2
  r = fma(0.5 * r, h, r);
  h = fma(-x * r, r, 1.0);
  return fma(0.5 * r, h, r);
}

// Huber kernel on s = |r|^2: rho, rho', rho''.  delta <= 0 or inf: plain least
// squares.  s == delta^2 takes the inlier branch.
__device__ __forceinline__ void huber(double s, double delta, double& rho, double& d1,
                                      double& d2) {
  if (delta > 0.0 && delta < 1e300 && s > delta * delta) {
    const double ir = rsqrt_nr(s);   // 1 / sqrt(s)
    rho = 2.0 * delta * (s * ir) - delta * delta;
    d1 = delta * ir;
    d2 = -0.5 * delta * ir * ir * ir;
  } else {
    rho = s;
    d1 = 1.0;
    d2 = 0.0;
  }
}

// Linearisation of one observation at (pose R, t | point p).
template <typename Real>
struct Lin {
  double rho_w;     // w * rho(s)
  double d1, d2;    // rho'(s), rho''(s)
  double wo;        // observation weight
  double X, Y, Z;   // camera-frame point
  Real r[2];        // residual pi(x_c) - o
  Real a0[3], a1[3];  // rows of A R_c (A = d pi / d x_c)
  Real xb[3];       // base-frame point
};

template <typename Real>
__device__ __forceinline__ Lin<Real> linearise(const double* __restrict__ xb, const double* C,
                                               double du, double dv, double wo, double delta) {
  Lin<Real> L;
  const double X = C[4] * xb[0] + C[5] * xb[1] + C[6] * xb[2] + C[13];
  const double Y = C[7] * xb[0] + C[8] * xb[1] + C[9] * xb[2] + C[14];
  const double Z = C[10] * xb[0] + C[11] * xb[1] + C[12] * xb[2] + C[15];
  const double iz = recip_nr(Z);
  const double xz = X * iz, yz = Y * iz;
  const double r0 = C[0] * xz - du, r1 = C[1] * yz - dv;
  const double s = r0 * r0 + r1 * r1;
  double rho, d1, d2;
  huber(s, delta, rho, d1, d2);
  L.rho_w = wo * rho;
  L.d1 = d1;
  L.d2 = d2;
  L.wo = wo;
  L.X = X;
  L.Y = Y;
  L.Z = Z;
  L.r[0] = (Real)r0;
  L.r[1] = (Real)r1;
  const double fi = C[0] * iz, gi = C[1] * iz;
  for (int c = 0; c < 3; ++c) {
    L.a0[c] = (Real)(fi * (C[4 + c] - xz * C[10 + c]));
    L.a1[c] = (Real)(gi * (C[7 + c] - yz * C[10 + c]));
    L.xb[c] = (Real)xb[c];
  }
  return L;
}

template <typename Real>
__device__ __forceinline__ void cross3(const Real* a, const Real* b, Real* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

// Lane shift by DPP (row_shr:n within rows of 16 lanes, row_bcast:15 / :31
// across rows) of a 32- or 64-bit value; lanes outside ROWMASK or without a
// source lane read `old`.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ int dpp_i(int old, int x) {
  return __builtin_amdgcn_update_dpp(old, x, CTRL, ROWMASK, 0xf, false);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dpp_r(float x) {
  return __int_as_float(dpp_i<CTRL, ROWMASK>(0, __float_as_int(x)));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_r(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = dpp_i<CTRL, ROWMASK>(0, (int)(b & 0xffffffffll));
  const int hi = dpp_i<CTRL, ROWMASK>(0, (int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Value of a double in lane `src` (wave-uniform) to every lane, by readlane.
__device__ __forceinline__ double wave_bcast(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// SE(3) exponential of xi = (rho, phi) as a 3x4 [R | t].  The coefficients
// A = sin(th)/th, B = (1 - cos th)/th^2, C = (th - sin th)/th^3 come from
// their power series in th^2 below th = 1 (nine terms: the first omitted one
// is under 1e-17, and the series has no cancellation), and from the closed
// forms above it.
__device__ __forceinline__ void exp_se3(const double* xi, double* T /*3x4*/) {
  const double rx = xi[0], ry = xi[1], rz = xi[2];
  const double px = xi[3], py = xi[4], pz = xi[5];
  const double th2 = px * px + py * py + pz * pz;
  double A, B, Cc;
  if (th2 < 1.0) {
    // A = 1 - t/(2*3) (1 - t/(4*5) (...)), B = (1 - t/(3*4) (...)) / 2,
    // C = (1 - t/(4*5) (...)) / 6, t = th^2
    double a = 1.0, b = 1.0, c = 1.0;
#pragma unroll
    for (int k = 8; k >= 0; --k) {
      const double n = 2.0 * k;
      a = fma(-th2 * (1.0 / ((n + 2.0) * (n + 3.0))), a, 1.0);
      b = fma(-th2 * (1.0 / ((n + 3.0) * (n + 4.0))), b, 1.0);
      c = fma(-th2 * (1.0 / ((n + 4.0) * (n + 5.0))), c, 1.0);
    }
    A = a;
    B = 0.5 * b;
    Cc = c / 6.0;
  } else {
    const double th = sqrt(th2);
    A = sin(th) / th;
    const double s = sin(0.5 * th);
    B = 2.0 * s * s / th2;
    Cc = (th - sin(th)) / (th2 * th);
  }
  const double K[9] = {0, -pz, py, pz, 0, -px, -py, px, 0};
  double K2[9];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      K2[3 * a + b] = K[3 * a] * K[b] + K[3 * a + 1] * K[3 + b] + K[3 * a + 2] * K[6 + b];
  double R[9], J[9];
  for (int k = 0; k < 9; ++k) {
    const double I = (k % 4 == 0) ? 1.0 : 0.0;
    R[k] = I + A * K[k] + B * K2[k];
    J[k] = I + B * K[k] + Cc * K2[k];
  }
  for (int a = 0; a < 3; ++a) {
    T[4 * a] = R[3 * a];
    T[4 * a + 1] = R[3 * a + 1];
    T[4 * a + 2] = R[3 * a + 2];
    T[4 * a + 3] = J[3 * a] * rx + J[3 * a + 1] * ry + J[3 * a + 2] * rz;
  }
}

}  // namespace ba
