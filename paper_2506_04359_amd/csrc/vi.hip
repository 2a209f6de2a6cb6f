// Visual-inertial window solve (paper Sec. 2.2, "Visual-Inertial", Eq. 9).
//
// The state of keyframe i is S_i = [T_i, v_i, b^a_i, b^w_i]; consecutive
// states are tied by an IMU factor built from the on-manifold preintegration
// of the samples between them (the model of Forster et al. 2017 that the
// paper cites).  The visual part of the window solve is unchanged; per LM
// attempt and window this file adds
//   k_vi_fac   one wave per IMU factor at the current state: residual,
//              Jacobian, J^T Lambda J and J^T Lambda r (FP64) into the
//              factor's record;
//   k_vi_lin   the pose-pose terms added into the summed reduced system and
//              the elimination of the extra variables y = (v, b^a, b^w) onto
//              the poses: A = H_yy + damping is block tridiagonal (9x9
//              blocks); with X = A^-1 H_yx and z = A^-1 g_y,
//                  S <- S - H_xy X,   rhs <- rhs + H_xy z,
//              so the reduced camera system keeps its size and the existing
//              Cholesky solves it;
//   k_vi_cand  after the poses' step dx: dy = -z - X dx, the candidate
//              velocities and biases, and the IMU cost at the candidate.
// Everything here is FP64 (a window has few IMU factors; their information
// matrices span many orders of magnitude).
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "device.hpp"
#include "geometry.hpp"
#include "vi.hpp"

namespace ba {
namespace {

// ---- SO(3) on 3x3 row-major matrices
__device__ void skew3(const double* v, double* K) {
  K[0] = 0.0;
  K[1] = -v[2];
  K[2] = v[1];
  K[3] = v[2];
  K[4] = 0.0;
  K[5] = -v[0];
  K[6] = -v[1];
  K[7] = v[0];
  K[8] = 0.0;
}

__device__ void mul33(const double* A, const double* B, double* C) {
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) C[3 * a + b] = A[3 * a] * B[b] + A[3 * a + 1] * B[3 + b] + A[3 * a + 2] * B[6 + b];
}

__device__ void mul33t(const double* A, const double* B, double* C) {   // A^T B
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) C[3 * a + b] = A[a] * B[b] + A[3 + a] * B[3 + b] + A[6 + a] * B[6 + b];
}

__device__ void mul3t3(const double* A, const double* B, double* C) {   // A B^T
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      C[3 * a + b] = A[3 * a] * B[3 * b] + A[3 * a + 1] * B[3 * b + 1] + A[3 * a + 2] * B[3 * b + 2];
}

__device__ void mv3(const double* A, const double* x, double* y) {
  for (int a = 0; a < 3; ++a) y[a] = A[3 * a] * x[0] + A[3 * a + 1] * x[1] + A[3 * a + 2] * x[2];
}

__device__ void mtv3(const double* A, const double* x, double* y) {   // A^T x
  for (int a = 0; a < 3; ++a) y[a] = A[a] * x[0] + A[3 + a] * x[1] + A[6 + a] * x[2];
}

// sin(th)/th, (1 - cos th)/th^2, (th - sin th)/th^3 (power series below th = 1)
__device__ void so3_coeffs(double th2, double& A, double& B, double& C) {
  if (th2 < 1.0) {
    double a = 1.0, b = 1.0, c = 1.0;
    for (int k = 8; k >= 0; --k) {
      const double n = 2.0 * k;
      a = fma(-th2 * (1.0 / ((n + 2.0) * (n + 3.0))), a, 1.0);
      b = fma(-th2 * (1.0 / ((n + 3.0) * (n + 4.0))), b, 1.0);
      c = fma(-th2 * (1.0 / ((n + 4.0) * (n + 5.0))), c, 1.0);
    }
    A = a;
    B = 0.5 * b;
    C = c / 6.0;
  } else {
    const double th = sqrt(th2);
    A = sin(th) / th;
    const double s = sin(0.5 * th);
    B = 2.0 * s * s / th2;
    C = (th - sin(th)) / (th2 * th);
  }
}

// Exp(phi) and the right Jacobian J_r(phi) = I - B K + C K^2.
__device__ void exp_so3_jr(const double* phi, double* R, double* Jr) {
  const double th2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  double A, B, C;
  so3_coeffs(th2, A, B, C);
  double K[9], K2[9];
  skew3(phi, K);
  mul33(K, K, K2);
  for (int k = 0; k < 9; ++k) {
    const double I = (k % 4 == 0) ? 1.0 : 0.0;
    R[k] = I + A * K[k] + B * K2[k];
    if (Jr) Jr[k] = I - B * K[k] + C * K2[k];
  }
}

// Log of a rotation (theta from atan2 of the antisymmetric and trace parts;
// the axis from the symmetric part near theta = pi).
__device__ void log_so3_33(const double* R, double* phi) {
  const double v[3] = {0.5 * (R[7] - R[5]), 0.5 * (R[2] - R[6]), 0.5 * (R[3] - R[1])};
  double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
  c = fmin(1.0, fmax(-1.0, c));
  const double s = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const double th = atan2(s, c);
  if (c > -0.999) {
    const double t2 = th * th;
    const double f = th < 1e-3 ? 1.0 + t2 * (1.0 / 6.0 + t2 * (7.0 / 360.0)) : th / s;
    for (int k = 0; k < 3; ++k) phi[k] = f * v[k];
    return;
  }
  const double Md[3] = {R[0] - c, R[4] - c, R[8] - c};
  int k = 0;
  if (Md[1] > Md[k]) k = 1;
  if (Md[2] > Md[k]) k = 2;
  const double ic = 1.0 / (1.0 - c);
  double a[3];
  a[k] = sqrt(fmax(Md[k] * ic, 0.0));
  const double ia = 1.0 / a[k];
  for (int m = 0; m < 3; ++m)
    if (m != k) a[m] = 0.5 * (R[3 * m + k] + R[3 * k + m]) * ic * ia;
  const double sg = (a[0] * v[0] + a[1] * v[1] + a[2] * v[2]) < 0.0 ? -1.0 : 1.0;
  for (int m = 0; m < 3; ++m) phi[m] = sg * th * a[m];
}

// J_r(phi)^-1 = I + K / 2 + d K^2, d = 1/th^2 - cot(th/2) / (2 th)
__device__ void jr_inv(const double* phi, double* Ji) {
  const double t2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
  double d;
  if (t2 < 1e-2) {
    d = 1.0 / 12.0 + t2 * (1.0 / 720.0 + t2 * (1.0 / 30240.0 + t2 * (1.0 / 1209600.0)));
  } else {
    const double th = sqrt(t2);
    d = 1.0 / t2 - cos(0.5 * th) / (sin(0.5 * th) * 2.0 * th);
  }
  double K[9], K2[9];
  skew3(phi, K);
  mul33(K, K, K2);
  for (int k = 0; k < 9; ++k) Ji[k] = ((k % 4 == 0) ? 1.0 : 0.0) + 0.5 * K[k] + d * K2[k];
}

// In-place Cholesky A = L L^T of an n x n row-major matrix (lower part
// written); false on a non-positive or non-finite pivot.
__device__ bool chol_n(double* A, int n) {
  for (int j = 0; j < n; ++j) {
    double d = A[n * j + j];
    for (int k = 0; k < j; ++k) d -= A[n * j + k] * A[n * j + k];
    if (!(d > 0.0) || !isfinite(d)) return false;
    const double l = sqrt(d);
    A[n * j + j] = l;
    const double il = 1.0 / l;
    for (int i = j + 1; i < n; ++i) {
      double v = A[n * i + j];
      for (int k = 0; k < j; ++k) v -= A[n * i + k] * A[n * j + k];
      A[n * i + j] = v * il;
    }
  }
  return true;
}

// y = L^-1 x and x = L^-T y for a Cholesky factor in the lower part of L (n x n)
__device__ void lsolve(const double* L, int n, double* x) {
  for (int i = 0; i < n; ++i) {
    double v = x[i];
    for (int k = 0; k < i; ++k) v -= L[n * i + k] * x[k];
    x[i] = v / L[n * i + i];
  }
}

__device__ void ltsolve(const double* L, int n, double* x) {
  for (int i = n - 1; i >= 0; --i) {
    double v = x[i];
    for (int k = i + 1; k < n; ++k) v -= L[n * k + i] * x[k];
    x[i] = v / L[n * i + i];
  }
}

// Residual (15) of the factor between states i and j and, with kJac, its
// Jacobian: 15 x 30 row-major, columns (rho_i, phi_i, v_i, b^a_i, b^w_i,
// rho_j, phi_j, v_j, b^a_j, b^w_j); only the non-zero entries are written (J
// must hold zeros).  pose: 3x4 base-from-world, st: v, b^a, b^w.
template <bool kJac>
__device__ void imu_factor(const double* Pi, const double* si, const double* Pj, const double* sj,
                           const double* pre, const double* g, double* r, double* J) {
  const double Ri[9] = {Pi[0], Pi[1], Pi[2], Pi[4], Pi[5], Pi[6], Pi[8], Pi[9], Pi[10]};
  const double Rj[9] = {Pj[0], Pj[1], Pj[2], Pj[4], Pj[5], Pj[6], Pj[8], Pj[9], Pj[10]};
  const double ti[3] = {Pi[3], Pi[7], Pi[11]}, tj[3] = {Pj[3], Pj[7], Pj[11]};
  double pi[3], pj[3];
  mtv3(Ri, ti, pi);
  mtv3(Rj, tj, pj);
  for (int k = 0; k < 3; ++k) {
    pi[k] = -pi[k];
    pj[k] = -pj[k];
  }
  const double* dR = pre + kPreDR;
  const double* JRg = pre + kPreJRg;
  double dbg[3], dba[3];
  for (int k = 0; k < 3; ++k) {
    dbg[k] = si[6 + k] - pre[kPreBg + k];
    dba[k] = si[3 + k] - pre[kPreBa + k];
  }
  double u[3], Eu[9], Jru[9], dRc[9];
  mv3(JRg, dbg, u);
  exp_so3_jr(u, Eu, Jru);
  mul33(dR, Eu, dRc);
  double RiRjT[9], E[9];
  mul3t3(Ri, Rj, RiRjT);          // R_i R_j^T
  mul33t(dRc, RiRjT, E);          // dRc^T R_i R_j^T
  double rR[3];
  log_so3_33(E, rR);
  const double dT = pre[kPreDT];
  double wv[3], wp[3];
  for (int k = 0; k < 3; ++k) {
    wv[k] = sj[k] - si[k] - g[k] * dT;
    wp[k] = pj[k] - pi[k] - si[k] * dT - 0.5 * g[k] * dT * dT;
  }
  double Riwv[3], Riwp[3];
  mv3(Ri, wv, Riwv);
  mv3(Ri, wp, Riwp);
  const double* Jvg = pre + kPreJvg;
  const double* Jva = pre + kPreJva;
  const double* Jpg = pre + kPreJpg;
  const double* Jpa = pre + kPreJpa;
  for (int a = 0; a < 3; ++a) {
    double cv = pre[kPreDv + a], cp = pre[kPreDp + a];
    for (int b = 0; b < 3; ++b) {
      cv += Jvg[3 * a + b] * dbg[b] + Jva[3 * a + b] * dba[b];
      cp += Jpg[3 * a + b] * dbg[b] + Jpa[3 * a + b] * dba[b];
    }
    r[a] = rR[a];
    r[3 + a] = Riwv[a] - cv;
    r[6 + a] = Riwp[a] - cp;
    r[9 + a] = sj[3 + a] - si[3 + a];
    r[12 + a] = sj[6 + a] - si[6 + a];
  }
  if (!kJac) return;
  double Jri[9];
  jr_inv(rR, Jri);
  double RjRiT[9], T1[9], T2[9], T3[9];
  mul3t3(Rj, Ri, RjRiT);
  mul33(Jri, RjRiT, T1);          // dr_R/dphi_i
  mul33t(E, Jru, T2);             // E^T J_r(u)
  mul33(T2, JRg, T3);             // E^T J_r(u) J_Rg
  double T4[9];
  mul33(Jri, T3, T4);
  double Kv[9], Kp[9];
  skew3(Riwv, Kv);
  skew3(Riwp, Kp);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      const int k = 3 * a + b;
      const double I = a == b ? 1.0 : 0.0;
      // r_R
      J[30 * a + 3 + b] = T1[k];
      J[30 * a + 12 + b] = -T4[k];
      J[30 * a + 18 + b] = -Jri[k];
      // r_v
      J[30 * (3 + a) + 3 + b] = -Kv[k];
      J[30 * (3 + a) + 6 + b] = -Ri[k];
      J[30 * (3 + a) + 9 + b] = -Jva[k];
      J[30 * (3 + a) + 12 + b] = -Jvg[k];
      J[30 * (3 + a) + 21 + b] = Ri[k];
      // r_p
      J[30 * (6 + a) + 0 + b] = I;
      J[30 * (6 + a) + 3 + b] = -Kp[k];
      J[30 * (6 + a) + 6 + b] = -Ri[k] * dT;
      J[30 * (6 + a) + 9 + b] = -Jpa[k];
      J[30 * (6 + a) + 12 + b] = -Jpg[k];
      J[30 * (6 + a) + 15 + b] = -RiRjT[k];
      // bias random walk
      if (a == b) {
        J[30 * (9 + a) + 9 + b] = -1.0;
        J[30 * (9 + a) + 24 + b] = 1.0;
        J[30 * (12 + a) + 12 + b] = -1.0;
        J[30 * (12 + a) + 27 + b] = 1.0;
      }
    }
}

__device__ double imu_cost1(const double* r, const double* Info) {
  double c = 0.0;
  for (int a = 0; a < 15; ++a) {
    double v = 0.0;
    for (int b = 0; b < 15; ++b) v += Info[15 * a + b] * r[b];
    c += r[a] * v;
  }
  return 0.5 * c;
}

}  // namespace

// ---------------------------------------------------------------------------
// preintegration: one thread per factor, samples in time order
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(64) void k_vi_preint(int n_factors, const int32_t* sample_begin, const double* gyro,
                                                  const double* accel, double dt, const double* bias_bar, double sg,
                                                  double sa, double sbg, double sba, double* out) {
  const int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= n_factors) return;
  double* pre = out + (size_t)kPreStride * f;
  const double ba[3] = {bias_bar[6 * f], bias_bar[6 * f + 1], bias_bar[6 * f + 2]};
  const double bg[3] = {bias_bar[6 * f + 3], bias_bar[6 * f + 4], bias_bar[6 * f + 5]};
  double dR[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, dv[3] = {0, 0, 0}, dp[3] = {0, 0, 0};
  double JRg[9] = {}, Jvg[9] = {}, Jva[9] = {}, Jpg[9] = {}, Jpa[9] = {};
  // covariance of the errors (dphi, dv, dp) in 3x3 blocks P_ij, i <= j
  double P00[9] = {}, P01[9] = {}, P02[9] = {}, P11[9] = {}, P12[9] = {}, P22[9] = {};
  const double qg = sg * sg / dt, qa = sa * sa / dt, h = 0.5 * dt;
  const int s0 = sample_begin[f], s1 = sample_begin[f + 1];
  for (int s = s0; s < s1; ++s) {
    double w[3], a[3];
    for (int k = 0; k < 3; ++k) {
      w[k] = (gyro[3 * s + k] - bg[k]) * dt;
      a[k] = accel[3 * s + k] - ba[k];
    }
    double Ek[9], Jr[9], Ax[9], dRAx[9];
    exp_so3_jr(w, Ek, Jr);
    skew3(a, Ax);
    mul33(dR, Ax, dRAx);
    // P <- A P A^T + noise with A = [[E^T, 0, 0], [B, I, 0], [B dt/2, dt I, I]]
    // and B = -dR [a]x dt: first T = A P by block rows, then T A^T
    double Bm[9];
    for (int k = 0; k < 9; ++k) Bm[k] = -dRAx[k] * dt;
    double T00[9], T01[9], T02[9], BP0[9], BP1[9], BP2[9];
    mul33t(Ek, P00, T00);
    mul33t(Ek, P01, T01);
    mul33t(Ek, P02, T02);
    mul33(Bm, P00, BP0);
    mul33(Bm, P01, BP1);
    mul33(Bm, P02, BP2);
    double T10[9], T11[9], T12[9], T20[9], T21[9], T22[9];
    for (int x = 0; x < 3; ++x)
      for (int y = 0; y < 3; ++y) {
        const int k = 3 * x + y, kt = 3 * y + x;   // P_10 = P_01^T, P_20 = P_02^T, P_21 = P_12^T
        T10[k] = BP0[k] + P01[kt];
        T11[k] = BP1[k] + P11[k];
        T12[k] = BP2[k] + P12[k];
        T20[k] = h * BP0[k] + dt * P01[kt] + P02[kt];
        T21[k] = h * BP1[k] + dt * P11[k] + P12[kt];
        T22[k] = h * BP2[k] + dt * P12[k] + P22[k];
      }
    double TB0[9], TB1[9], TB2[9];
    mul33(T00, Ek, P00);
    mul3t3(T00, Bm, TB0);
    mul3t3(T10, Bm, TB1);
    mul3t3(T20, Bm, TB2);
    for (int k = 0; k < 9; ++k) {
      P01[k] = TB0[k] + T01[k];
      P02[k] = h * TB0[k] + dt * T01[k] + T02[k];
      P11[k] = TB1[k] + T11[k];
      P12[k] = h * TB1[k] + dt * T11[k] + T12[k];
      P22[k] = h * TB2[k] + dt * T21[k] + T22[k];
    }
    // gyroscope noise through J_r dt, accelerometer noise through dR dt and dR dt^2 / 2
    for (int x = 0; x < 3; ++x)
      for (int y = 0; y < 3; ++y) {
        double gg = 0.0, aa = 0.0;
        for (int k = 0; k < 3; ++k) {
          gg += Jr[3 * x + k] * Jr[3 * y + k];
          aa += dR[3 * x + k] * dR[3 * y + k];
        }
        P00[3 * x + y] += qg * dt * dt * gg;
        P11[3 * x + y] += qa * dt * dt * aa;
        P12[3 * x + y] += qa * 0.5 * dt * dt * dt * aa;
        P22[3 * x + y] += qa * 0.25 * dt * dt * dt * dt * aa;
      }
    // bias Jacobians (with dR, dv, J_Rg before this sample's update)
    double M1[9];
    mul33(dRAx, JRg, M1);
    for (int k = 0; k < 9; ++k) {
      Jpa[k] += Jva[k] * dt - 0.5 * dR[k] * dt * dt;
      Jpg[k] += Jvg[k] * dt - 0.5 * M1[k] * dt * dt;
      Jva[k] -= dR[k] * dt;
      Jvg[k] -= M1[k] * dt;
    }
    double EtJ[9];
    mul33t(Ek, JRg, EtJ);
    for (int k = 0; k < 9; ++k) JRg[k] = EtJ[k] - Jr[k] * dt;
    // the measurement
    double dRa[3];
    mv3(dR, a, dRa);
    for (int k = 0; k < 3; ++k) {
      dp[k] += dv[k] * dt + 0.5 * dRa[k] * dt * dt;
      dv[k] += dRa[k] * dt;
    }
    double nR[9];
    mul33(dR, Ek, nR);
    for (int k = 0; k < 9; ++k) dR[k] = nR[k];
  }
  const double dT = dt * (s1 - s0);
  for (int k = 0; k < 9; ++k) {
    pre[kPreDR + k] = dR[k];
    pre[kPreJRg + k] = JRg[k];
    pre[kPreJvg + k] = Jvg[k];
    pre[kPreJva + k] = Jva[k];
    pre[kPreJpg + k] = Jpg[k];
    pre[kPreJpa + k] = Jpa[k];
  }
  for (int k = 0; k < 3; ++k) {
    pre[kPreDv + k] = dv[k];
    pre[kPreDp + k] = dp[k];
    pre[kPreBa + k] = ba[k];
    pre[kPreBg + k] = bg[k];
  }
  pre[kPreDT] = dT;
  // information: the inverse of the 9x9 covariance (Cholesky), the bias
  // random walk 1 / (sigma^2 dT).  One sample's covariance has rank 6 (the
  // same accelerometer noise moves velocity and position), so an interval of
  // fewer than two samples gets NaN information.
  double* Info = pre + kPreInfo;
  for (int k = 0; k < 225; ++k) Info[k] = 0.0;
  double cov[81];
  for (int x = 0; x < 3; ++x)
    for (int y = 0; y < 3; ++y) {
      const int k = 3 * x + y, kt = 3 * y + x;
      cov[9 * x + y] = P00[k];
      cov[9 * x + 3 + y] = P01[k];
      cov[9 * x + 6 + y] = P02[k];
      cov[9 * (3 + x) + y] = P01[kt];
      cov[9 * (3 + x) + 3 + y] = P11[k];
      cov[9 * (3 + x) + 6 + y] = P12[k];
      cov[9 * (6 + x) + y] = P02[kt];
      cov[9 * (6 + x) + 3 + y] = P12[kt];
      cov[9 * (6 + x) + 6 + y] = P22[k];
    }
  const bool ok = s1 - s0 >= 2 && chol_n(cov, 9);
  for (int c = 0; c < 9; ++c) {
    double e[9] = {};
    e[c] = 1.0;
    if (ok) {
      lsolve(cov, 9, e);
      ltsolve(cov, 9, e);
    } else {
      for (int k = 0; k < 9; ++k) e[k] = __builtin_nan("");
    }
    for (int k = 0; k < 9; ++k) Info[15 * k + c] = e[k];
  }
  for (int k = 0; k < 3; ++k) {
    Info[15 * (9 + k) + 9 + k] = 1.0 / (sba * sba * dT);
    Info[15 * (12 + k) + 12 + k] = 1.0 / (sbg * sbg * dT);
  }
}

// ---------------------------------------------------------------------------
// IMU factors at the current state: one wave per factor
// ---------------------------------------------------------------------------

// Factor record in the workspace: H = J^T Lambda J (30 x 30), g = J^T Lambda r
// (30), r (15) and the factor's cost.
constexpr int kFH = 0, kFg = 900, kFr = 930, kFc = 945, kFRec = 946;
static_assert(kFRec <= kViFactorStride, "factor record stride");

__global__ __launch_bounds__(64) void k_vi_fac(ViArgs V, int wbase) {
  __shared__ double sJ[450], sLJ[450], sI[225], sr[15];
  const int wi = V.win_order[wbase + blockIdx.y];
  const WinDev W = V.win[wi];
  const int f = blockIdx.x, lane = threadIdx.x;
  if (f >= W.n_poses - 1) return;
  const int cur = V.state[wi].cur;
  const double* poses = (cur ? V.poses_b : V.poses) + 12 * W.pose_off;
  const double* states = (cur ? V.states_b : V.states) + 9 * W.pose_off;
  const double* pre = V.preint + (size_t)kPreStride * f;
  double* F = V.rec + (size_t)kViFactorStride * f;
  for (int e = lane; e < 450; e += 64) sJ[e] = 0.0;
  for (int e = lane; e < 225; e += 64) sI[e] = pre[kPreInfo + e];
  __syncthreads();
  if (lane == 0) {
    double r[15];
    imu_factor<true>(poses + 12 * f, states + 9 * f, poses + 12 * (f + 1), states + 9 * (f + 1), pre, V.g, r, sJ);
    for (int k = 0; k < 15; ++k) sr[k] = r[k];
  }
  __syncthreads();
  // Lambda J (15 x 30)
  for (int e = lane; e < 450; e += 64) {
    const int a = e / 30, c = e % 30;
    double v = 0.0;
    for (int k = 0; k < 15; ++k) v += sI[15 * a + k] * sJ[30 * k + c];
    sLJ[e] = v;
  }
  __syncthreads();
  // H and g in one pass over the record's first 930 doubles
  for (int e = lane; e < 930; e += 64) {
    double v = 0.0;
    if (e < 900) {
      const int a = e / 30, c = e % 30;
      for (int k = 0; k < 15; ++k) v += sJ[30 * k + a] * sLJ[30 * k + c];
    } else {
      for (int k = 0; k < 15; ++k) v += sLJ[30 * k + e - 900] * sr[k];
    }
    F[e] = v;
  }
  if (lane < 15) F[kFr + lane] = sr[lane];
  if (lane == 0) F[kFc] = imu_cost1(sr, sI);
}

// ---------------------------------------------------------------------------
// elimination of the extra variables onto the poses: one workgroup per window
// ---------------------------------------------------------------------------

// H_xy of factor f staged as 12 x 18: rows (x_i, x_j) are H rows 0..5 and
// 15..20, columns (y_i, y_j) are H columns 6..14 and 21..29.
__device__ inline int hx_row(int q) { return q < 6 ? q : 9 + q; }
__device__ inline int hy_col(int c) { return c < 9 ? 6 + c : 12 + c; }

// Cholesky of a 9x9 block held in registers (lower part), the pivots by the
// refined rsqrt: L_jj = d rsqrt(d) and inv_j = rsqrt(d) (no square root or
// division on the pivot chain).  False on a non-positive or non-finite pivot.
__device__ __forceinline__ bool chol9_regs(double (&A)[81], double (&inv)[9]) {
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    double d = A[10 * j];
#pragma unroll
    for (int k = 0; k < j; ++k) d -= A[9 * j + k] * A[9 * j + k];
    if (!(d > 0.0) || !isfinite(d)) return false;
    const double ir = rsqrt(d);
    A[10 * j] = d * ir;
    inv[j] = ir;
#pragma unroll
    for (int i = j + 1; i < 9; ++i) {
      double v = A[9 * i + j];
#pragma unroll
      for (int k = 0; k < j; ++k) v -= A[9 * i + k] * A[9 * j + k];
      A[9 * i + j] = v * ir;
    }
  }
  return true;
}

// Waits for the LDS reads that produced v before anything that uses v (the
// reads are issued together and waited for once).
template <int N>
__device__ __forceinline__ void vi_lds_fence(double (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) __asm__ volatile("" : "+v"(v[i]));
}

// A 9x9 Cholesky factor's strictly lower entries (row i, column k < i at
// i (i - 1) / 2 + k) and reciprocal diagonal, read from LDS together and
// waited for once, then the two triangular solves on registers.
struct L9 {
  double l[36], inv[9];
};
__device__ __forceinline__ void load_l9(const double* L, const double* inv, L9& F) {
#pragma unroll
  for (int i = 1, q = 0; i < 9; ++i)
#pragma unroll
    for (int k = 0; k < i; ++k, ++q) F.l[q] = L[9 * i + k];
#pragma unroll
  for (int i = 0; i < 9; ++i) F.inv[i] = inv[i];
  vi_lds_fence(F.l);
  vi_lds_fence(F.inv);
}
__device__ __forceinline__ void lsolve9r(const L9& F, double (&x)[9]) {
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    double v = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) v -= F.l[i * (i - 1) / 2 + k] * x[k];
    x[i] = v * F.inv[i];
  }
}
__device__ __forceinline__ void ltsolve9r(const L9& F, double (&x)[9]) {
#pragma unroll
  for (int i = 8; i >= 0; --i) {
    double v = x[i];
#pragma unroll
    for (int k = i + 1; k < 9; ++k) v -= F.l[k * (k - 1) / 2 + i] * x[k];
    x[i] = v * F.inv[i];
  }
}

constexpr int kViLinThreads = 256;   // threads of the elimination workgroup

template <bool XL>
__global__ __launch_bounds__(kViLinThreads) void k_vi_lin(ViArgs V, int wbase) {
  extern __shared__ __align__(16) double sXd[];     // X when it fits in LDS (XL)
  __shared__ double sA[kViMaxStates * 81];          // A_kk (damped), then its Cholesky factor L_k
  __shared__ double sO[(kViMaxStates - 1) * 81];    // A_{k,k+1}
  __shared__ double sC[kViMaxStates * 81];          // C_k = A_{k,k-1} L_{k-1}^-T, k >= 1
  __shared__ double sH[(kViMaxStates - 1) * 216];   // H_xy per factor
  __shared__ double sG[kViMaxStates * 9];           // g_y
  __shared__ double sInv[kViMaxStates * 9];         // 1 / diag(L_k)
  __shared__ int sPose[kViMaxStates];               // pose of each free slot
  __shared__ int sOk;
  const int wi = V.win_order[wbase + blockIdx.x];
  const WinDev W = V.win[wi];
  const WinState& st = V.state[wi];
  const int tid = threadIdx.x;
  const int N = W.n_poses, nf = N - 1, nS = 6 * W.n_free, ncol = nS + 1;
  const double* F = V.rec;                           // per factor records
  // 9N x (nS + 1): A^-1 H_yx, then z = A^-1 g_y; worked on in LDS when it
  // fits (XL) and copied out at the end, since k_vi_cand reads it
  double* Xg = V.rec + (size_t)kViFactorStride * nf;
  double* X = XL ? sXd : Xg;
  const int* fs = V.free_slot + W.pose_off;
  if (tid < N && fs[tid] >= 0) sPose[fs[tid]] = tid;
  if (tid == 0) sOk = 1;
  // 1. stage A = H_yy + damping (block tridiagonal), A_{k,k+1}, H_xy and g_y:
  //    one index space over the four arrays, eight elements per thread and
  //    round, a round's reads (two per element, unconditional: an unused one
  //    reads F[0]) all in flight before its first LDS store
  const double lam = st.lambda;
  {
    const int nA = N * 81, nO = nf * 81, nH = nf * 216, nG = N * 9, ntot = nA + nO + nH + nG;
    constexpr int R = 8;
    for (int base = 0; base < ntot; base += R * blockDim.x) {
      long long i0[R], i1[R];
      double v0[R], v1[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = base + tid + r * (int)blockDim.x;
        i0[r] = -1;
        i1[r] = -1;
        if (e < nA) {
          const int k = e / 81, x = (e % 81) / 9, y = e % 9;
          if (k >= 1) i0[r] = (long long)kViFactorStride * (k - 1) + kFH + 30 * (21 + x) + 21 + y;
          if (k < nf) i1[r] = (long long)kViFactorStride * k + kFH + 30 * (6 + x) + 6 + y;
        } else if (e < nA + nO) {
          const int t = e - nA, f = t / 81, x = (t % 81) / 9, y = t % 9;
          i0[r] = (long long)kViFactorStride * f + kFH + 30 * (6 + x) + 21 + y;
        } else if (e < nA + nO + nH) {
          const int t = e - nA - nO, f = t / 216, q = (t % 216) / 18, c = t % 18;
          i0[r] = (long long)kViFactorStride * f + kFH + 30 * hx_row(q) + hy_col(c);
        } else if (e < ntot) {
          const int t = e - nA - nO - nH, k = t / 9, x = t % 9;
          if (k >= 1) i0[r] = (long long)kViFactorStride * (k - 1) + kFg + 21 + x;
          if (k < nf) i1[r] = (long long)kViFactorStride * k + kFg + 6 + x;
        }
        v0[r] = F[i0[r] >= 0 ? i0[r] : 0];
        v1[r] = F[i1[r] >= 0 ? i1[r] : 0];
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = base + tid + r * (int)blockDim.x;
        double v = 0.0;
        if (i0[r] >= 0) v += v0[r];
        if (i1[r] >= 0) v += v1[r];
        if (e < nA) {
          const int x = (e % 81) / 9, y = e % 9;
          if (x == y) v += lam * fmax(v, 1e-9);
          sA[e] = v;
        } else if (e < nA + nO) {
          sO[e - nA] = v;
        } else if (e < nA + nO + nH) {
          sH[e - nA - nO] = v;
        } else if (e < ntot) {
          sG[e - nA - nO - nH] = v;
        }
      }
    }
  }
  // 2. the IMU cost at the current state (fixed order), for the first attempt
  if (tid == 0) {
    double cf[kViMaxStates - 1];   // every factor's cost read before the sum
#pragma unroll
    for (int f = 0; f < kViMaxStates - 1; ++f) cf[f] = f < nf ? F[(size_t)kViFactorStride * f + kFc] : 0.0;
    double c = 0.0;
#pragma unroll
    for (int f = 0; f < kViMaxStates - 1; ++f)
      if (f < nf) c += cf[f];
    V.cost_a[wi] = c;
  }
  // pose-pose terms into the summed reduced system: upper entries of the
  // diagonal blocks, whole off-diagonal blocks (a, a + 1), -g into the rhs,
  // the diagonal into diag(U) (the damping uses the whole diagonal); every
  // read of a thread's elements goes out before its first update
  const int nblk = W.n_free * (W.n_free + 1) / 2;
  double* S = V.ssum + W.sum_off;
  double* sB = S + nblk * kBS;   // the reduced right-hand side (global)
  for (int base = 0; base < N * 36; base += 2 * blockDim.x) {
    double fv[2][5], sv[2][4];
    long long so[2][4];
    int sa_[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = base + tid + r * (int)blockDim.x;
      const bool in = e < N * 36;
      const int a = in ? e / 36 : 0, rr = (e % 36) / 6, c = e % 6;
      const int sa = in ? fs[a] : -1;
      sa_[r] = sa;
      // F reads: diagonal-block terms of factors a - 1 and a, the off-diagonal
      // block of factor a, the rhs terms of factors a - 1 and a
      const long long fo[5] = {
          a >= 1 ? (long long)kViFactorStride * (a - 1) + kFH + 30 * (15 + rr) + 15 + c : 0,
          a < nf ? (long long)kViFactorStride * a + kFH + 30 * rr + c : 0,
          a < nf ? (long long)kViFactorStride * a + kFH + 30 * rr + 15 + c : 0,
          a >= 1 ? (long long)kViFactorStride * (a - 1) + kFg + 15 + rr : 0,
          a < nf ? (long long)kViFactorStride * a + kFg + rr : 0};
#pragma unroll
      for (int q = 0; q < 5; ++q) fv[r][q] = F[fo[q]];
      const int sb = (sa >= 0 && a < nf) ? fs[a + 1] : -1;
      so[r][0] = sa >= 0 && c >= rr ? (long long)kBS * blk_index(sa, sa, W.n_free) + 6 * rr + c : -1;
      so[r][1] = sa >= 0 && sb >= 0 ? (long long)kBS * blk_index(sa, sb, W.n_free) + 6 * rr + c : -1;
      so[r][2] = sa >= 0 && c == 0 ? (long long)(nblk * kBS + 6 * sa + rr) : -1;
      so[r][3] = sa >= 0 && c == rr ? (long long)(nblk * kBS + nS + 6 * sa + rr) : -1;
#pragma unroll
      for (int q = 0; q < 4; ++q) sv[r][q] = S[so[r][q] >= 0 ? so[r][q] : 0];
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = base + tid + r * (int)blockDim.x;
      const int sa = sa_[r];
      if (e >= N * 36 || sa < 0) continue;
      const int a = e / 36, rr = (e % 36) / 6, c = e % 6;
      double v = 0.0;
      if (a >= 1) v += fv[r][0];
      if (a < nf) v += fv[r][1];
      if (so[r][0] >= 0) S[so[r][0]] = sv[r][0] + v;
      if (so[r][3] >= 0) S[so[r][3]] = sv[r][3] + v;
      if (so[r][1] >= 0) S[so[r][1]] = sv[r][1] + fv[r][2];
      if (so[r][2] >= 0) {
        double gg = 0.0;
        if (a >= 1) gg += fv[r][3];
        if (a < nf) gg += fv[r][4];
        S[so[r][2]] = sv[r][2] - gg;
      }
    }
  }
  __syncthreads();
  // 3. block tridiagonal Cholesky of A, state by state
  for (int k = 0; k < N; ++k) {
    if (k >= 1) {
      if (tid < 9) {   // row tid of C_k: L_{k-1} c = column tid of A_{k-1,k}
        L9 F;
        load_l9(sA + 81 * (k - 1), sInv + 9 * (k - 1), F);
        double row[9];
#pragma unroll
        for (int y = 0; y < 9; ++y) row[y] = sO[81 * (k - 1) + 9 * y + tid];
        vi_lds_fence(row);
        lsolve9r(F, row);
#pragma unroll
        for (int y = 0; y < 9; ++y) sC[81 * k + 9 * tid + y] = row[y];
      }
      __syncthreads();
      if (tid < 81) {
        const int x = tid / 9, y = tid % 9;
        double v = 0.0;
        for (int m = 0; m < 9; ++m) v += sC[81 * k + 9 * x + m] * sC[81 * k + 9 * y + m];
        sA[81 * k + tid] -= v;
      }
      __syncthreads();
    }
    if (tid == 0) {
      double Ak[81], iv[9];
#pragma unroll
      for (int e = 0; e < 81; ++e) Ak[e] = sA[81 * k + e];
      vi_lds_fence(Ak);
      if (chol9_regs(Ak, iv)) {
#pragma unroll
        for (int e = 0; e < 81; ++e) sA[81 * k + e] = Ak[e];
#pragma unroll
        for (int x = 0; x < 9; ++x) sInv[9 * k + x] = iv[x];
      } else {
        sOk = 0;
      }
    }
    __syncthreads();
    if (!sOk) break;
  }
  if (!sOk) {
    if (tid == 0) V.part_flag_a[W.chunk_begin] = 1;   // the reduce rejects the attempt
    return;
  }
  // 4. X = A^-1 [H_yx | g_y] by a forward sweep w_k = L_k^-1 (u_k - C_k w_{k-1})
  //    and a backward sweep u_k = L_k^-T (w_k - C_{k+1}^T u_{k+1}) over the
  //    states, all columns at once: per state, the coupling product (one
  //    entry per thread) and then the triangular solve (one column per
  //    thread), a barrier after each.  Columns above a pose's first state
  //    stay exactly zero.  sO (A_{k,k+1}) is no longer needed and holds the
  //    9 x ncol products.
  double* sT = sO;
  auto u_entry = [&](int k, int x, int col) -> double {
    double v = 0.0;
    if (col == nS) {
      v = sG[9 * k + x];
    } else {
      // factor a - 1 holds pose a as x_j (rows 6 + r), factor a as x_i (rows r)
      const int a = sPose[col / 6], r = col % 6;
      if (a >= 1 && k == a - 1) v += sH[216 * (a - 1) + 18 * (6 + r) + x];
      if (a >= 1 && k == a) v += sH[216 * (a - 1) + 18 * (6 + r) + 9 + x];
      if (a < nf && k == a) v += sH[216 * a + 18 * r + x];
      if (a < nf && k == a + 1) v += sH[216 * a + 18 * r + 9 + x];
    }
    return v;
  };
  for (int k = 0; k < N; ++k) {
    for (int e = tid; e < 9 * ncol; e += blockDim.x) {
      const int x = e / ncol, col = e - ncol * x;
      double v = u_entry(k, x, col);
      if (k >= 1) {
        double c[9], wp[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) {
          c[m] = sC[81 * k + 9 * x + m];
          wp[m] = X[(size_t)ncol * (9 * (k - 1) + m) + col];
        }
        vi_lds_fence(c);
        vi_lds_fence(wp);
#pragma unroll
        for (int m = 0; m < 9; ++m) v -= c[m] * wp[m];
      }
      sT[e] = v;
    }
    __syncthreads();
    for (int col = tid; col < ncol; col += blockDim.x) {
      L9 F;
      load_l9(sA + 81 * k, sInv + 9 * k, F);
      double w[9];
#pragma unroll
      for (int x = 0; x < 9; ++x) w[x] = sT[ncol * x + col];
      vi_lds_fence(w);
      lsolve9r(F, w);
#pragma unroll
      for (int x = 0; x < 9; ++x) X[(size_t)ncol * (9 * k + x) + col] = w[x];
    }
    __syncthreads();
  }
  for (int k = N - 1; k >= 0; --k) {
    for (int e = tid; e < 9 * ncol; e += blockDim.x) {
      const int x = e / ncol, col = e - ncol * x;
      double t = X[(size_t)ncol * (9 * k + x) + col];
      if (k + 1 < N) {
        double c[9], un[9];
#pragma unroll
        for (int m = 0; m < 9; ++m) {
          c[m] = sC[81 * (k + 1) + 9 * m + x];
          un[m] = X[(size_t)ncol * (9 * (k + 1) + m) + col];
        }
        vi_lds_fence(c);
        vi_lds_fence(un);
#pragma unroll
        for (int m = 0; m < 9; ++m) t -= c[m] * un[m];
      }
      sT[e] = t;
    }
    __syncthreads();
    for (int col = tid; col < ncol; col += blockDim.x) {
      L9 F;
      load_l9(sA + 81 * k, sInv + 9 * k, F);
      double v[9];
#pragma unroll
      for (int x = 0; x < 9; ++x) v[x] = sT[ncol * x + col];
      vi_lds_fence(v);
      ltsolve9r(F, v);
#pragma unroll
      for (int x = 0; x < 9; ++x) X[(size_t)ncol * (9 * k + x) + col] = v[x];
    }
    __syncthreads();
  }
  // 5. S <- S - H_xy X (upper blocks), rhs <- rhs + H_xy z; one row of a block
  //    (or of the rhs) per task
  auto hxy = [&](int a, int r, int k, int x) -> double {   // H(x_a row r, y_k component x)
    double v = 0.0;
    if (a >= 1 && (k == a - 1 || k == a)) v += sH[216 * (a - 1) + 18 * (6 + r) + (k == a - 1 ? x : 9 + x)];
    if (a < nf && (k == a || k == a + 1)) v += sH[216 * a + 18 * r + (k == a ? x : 9 + x)];
    return v;
  };
  for (int e = tid; e < (nblk + W.n_free) * 6; e += blockDim.x) {
    const int b = e / 6, r = e % 6;
    int sa, sb = 0;
    const bool rhs = b >= nblk;
    if (rhs)
      sa = b - nblk;
    else
      upper_pair(b, W.n_free, sa, sb);
    const int a = sPose[sa];
    const int k1 = a + 1 < N ? a + 1 : N - 1;
    if (rhs) {
      double v = 0.0;
      for (int k = (a >= 1 ? a - 1 : 0); k <= k1; ++k)
        for (int x = 0; x < 9; ++x) v += hxy(a, r, k, x) * X[(size_t)ncol * (9 * k + x) + nS];
      sB[6 * sa + r] += v;
      continue;
    }
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int k = (a >= 1 ? a - 1 : 0); k <= k1; ++k)
      for (int x = 0; x < 9; ++x) {
        const double h = hxy(a, r, k, x);
        const double* xr = X + (size_t)ncol * (9 * k + x) + 6 * sb;
        for (int c = 0; c < 6; ++c) acc[c] += h * xr[c];
      }
    for (int c = (sa == sb ? r : 0); c < 6; ++c) S[kBS * b + 6 * r + c] -= acc[c];
  }
  if (XL)
    for (int e = tid; e < 9 * N * ncol; e += blockDim.x) Xg[e] = sXd[e];
}

// ---------------------------------------------------------------------------
// candidate velocities and biases, the IMU cost at the candidate
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_vi_cand(ViArgs V, int wbase) {
  const int wi = V.win_order[wbase + blockIdx.x];
  const WinDev W = V.win[wi];
  const WinState& st = V.state[wi];
  const int tid = threadIdx.x;
  if (st.fail) {
    if (tid == 0) V.cost_b[wi] = 0.0;
    return;
  }
  const int N = W.n_poses, nf = N - 1, nS = 6 * W.n_free, ncol = nS + 1;
  const int cur = st.cur;
  const double* states = (cur ? V.states_b : V.states) + 9 * W.pose_off;
  double* cstates = (cur ? V.states : V.states_b) + 9 * W.pose_off;
  const double* cposes = (cur ? V.poses : V.poses_b) + 12 * W.pose_off;
  const double* X = V.rec + (size_t)kViFactorStride * nf;
  const double* dx = V.dp + kDpStride * wi;
  // dy = -z - X dx
  for (int e = tid; e < 9 * N; e += blockDim.x) {
    double v = -X[(size_t)ncol * e + nS];
    for (int c = 0; c < nS; ++c) v -= X[(size_t)ncol * e + c] * dx[c];
    cstates[e] = states[e] + v;
  }
  __syncthreads();
  __shared__ double sc[kViMaxStates];
  const double* pre = V.preint;
  for (int f = tid; f < nf; f += blockDim.x) {
    double r[15];
    imu_factor<false>(cposes + 12 * f, cstates + 9 * f, cposes + 12 * (f + 1), cstates + 9 * (f + 1),
                      pre + (size_t)kPreStride * f, V.g, r, nullptr);
    sc[f] = imu_cost1(r, pre + (size_t)kPreStride * f + kPreInfo);
  }
  __syncthreads();
  if (tid == 0) {
    double c = 0.0;
    for (int f = 0; f < nf; ++f) c += sc[f];
    V.cost_b[wi] = c;
  }
}

hipError_t launch_vi_preint(int n_factors, const int32_t* sample_begin, const double* gyro, const double* accel,
                            double dt, const double* bias_bar, const double* noise, double* out, hipStream_t st) {
  if (n_factors <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_vi_preint, dim3((n_factors + 63) / 64), dim3(64), 0, st, n_factors, sample_begin, gyro,
                     accel, dt, bias_bar, noise[0], noise[1], noise[2], noise[3], out);
  return hipGetLastError();
}

void launch_vi_lin(const ViArgs& V, int wbase, int nwin, hipStream_t st) {
  if (nwin <= 0 || V.max_factors <= 0) return;
  hipLaunchKernelGGL(k_vi_fac, dim3(V.max_factors, nwin), dim3(64), 0, st, V, wbase);
  // X (9N x (6 n_free + 1) doubles, n_free <= N) in LDS beside the static
  // arrays when the CU's 160 KB hold both.  The static size is the compiled
  // kernel's own (asked once per process, when its dynamic LDS limit is
  // raised, as for the other kernels); if either call fails, X stays in the
  // workspace.
  constexpr size_t kLds = 160 * 1024;
  const int N = V.max_factors + 1;
  const size_t xb = sizeof(double) * 9 * (size_t)N * (6 * (size_t)N + 1);
  static std::once_flag once;
  static bool attr = false;
  static size_t kStatic = kLds;
  std::call_once(once, [] {
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, reinterpret_cast<const void*>(&k_vi_lin<true>)) != hipSuccess ||
        fa.sharedSizeBytes >= kLds)
      return;
    kStatic = fa.sharedSizeBytes;
    attr = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vi_lin<true>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)(kLds - kStatic)) == hipSuccess;
  });
  if (attr && kStatic + xb <= kLds)
    hipLaunchKernelGGL(k_vi_lin<true>, dim3(nwin), dim3(kViLinThreads), xb, st, V, wbase);
  else
    hipLaunchKernelGGL(k_vi_lin<false>, dim3(nwin), dim3(kViLinThreads), 0, st, V, wbase);
}

void launch_vi_cand(const ViArgs& V, int wbase, int nwin, hipStream_t st) {
  if (nwin > 0) hipLaunchKernelGGL(k_vi_cand, dim3(nwin), dim3(256), 0, st, V, wbase);
}

}  // namespace ba
