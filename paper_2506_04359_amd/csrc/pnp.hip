// gfx950 motion-only bundle adjustment: many independent frames, each one pose
// refined against fixed landmarks (paper Sec. 2.2: stereo pose estimation,
// Eq. 4; the multi-camera rig, Eq. 6; the loop-closure relative pose against
// landmarks moved into a map frame by a known T^mw, Eq. 14).
//
// One wave per frame runs every LM attempt of that frame inside one launch (the
// frames share nothing, so no grid-wide step is needed):
//   linearise  lanes stride over the frame's observations: FP64 transform and
//              residual, Huber weight, 2x6 pose Jacobian, U (21) and g (6)
//              accumulated per lane (FP32 in mixed mode), then summed over the
//              wave in FP64 by DPP
//   solve      every lane: (U + lambda diag(max(U_kk, 1e-9))) d = -g by a 6x6
//              FP64 Cholesky; a non-positive pivot rejects the attempt
//   candidate  T' = Exp(d) T (FP64); lanes re-project every observation: any
//              depth <= min_depth rejects, else the robust cost in FP64
//   accept     F' < F (strict): T <- T', lambda / 10; else lambda x 10
// The linearisation is redone only after an accepted step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.hpp"
#include "geometry.hpp"
#include "pnp.hpp"

namespace ba {

constexpr int kPnpWaves = 4;   // frames per workgroup

// Sum over the wave (inclusive DPP scan, total read from lane 63).
__device__ __forceinline__ double wave_total(double v) {
  v += dpp_r<0x111, 0xf>(v);   // row_shr:1
  v += dpp_r<0x112, 0xf>(v);   // row_shr:2
  v += dpp_r<0x114, 0xf>(v);   // row_shr:4
  v += dpp_r<0x118, 0xf>(v);   // row_shr:8
  v += dpp_r<0x142, 0xa>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_r<0x143, 0xc>(v);   // row_bcast:31 into rows 2 and 3
  return wave_bcast(v, 63);
}

// x_b = T (M p) of one landmark (M = the frame's map-from-world or identity).
__device__ __forceinline__ void frame_point(const double* T, const double* M, bool has_m,
                                            const double* p, double* xb) {
  double q[3] = {p[0], p[1], p[2]};
  if (has_m) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
      q[a] = M[4 * a] * p[0] + M[4 * a + 1] * p[1] + M[4 * a + 2] * p[2] + M[4 * a + 3];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
    xb[a] = T[4 * a] * q[0] + T[4 * a + 1] * q[1] + T[4 * a + 2] * q[2] + T[4 * a + 3];
}

// Upper Cholesky solve of the damped 6x6 system (packed upper U, row-major):
// x = -(U + lam diag(max(U_kk, 1e-9)))^-1 g.  False on a non-positive or
// non-finite pivot.
__device__ __forceinline__ bool solve6(const double* U, const double* g, double lam, double* x) {
  double A[36];
  int e = 0;
#pragma unroll
  for (int r = 0; r < 6; ++r)
#pragma unroll
    for (int c = r; c < 6; ++c, ++e) {
      A[6 * r + c] = U[e];
      A[6 * c + r] = U[e];
    }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double d = A[7 * k];
    A[7 * k] = d + lam * (d > 1e-9 ? d : 1e-9);
  }
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    double d = A[7 * a];
#pragma unroll
    for (int m = 0; m < a; ++m) d -= A[6 * m + a] * A[6 * m + a];
    if (!(d > 0.0) || !isfinite(d)) return false;
    const double ra = sqrt(d);
    A[7 * a] = ra;
    const double ir = 1.0 / ra;
#pragma unroll
    for (int c = a + 1; c < 6; ++c) {
      double v = A[6 * a + c];
#pragma unroll
      for (int m = 0; m < a; ++m) v -= A[6 * m + a] * A[6 * m + c];
      A[6 * a + c] = v * ir;
    }
  }
  double y[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) {   // R^T y = -g
    double v = -g[a];
#pragma unroll
    for (int m = 0; m < a; ++m) v -= A[6 * m + a] * y[m];
    y[a] = v / A[7 * a];
  }
#pragma unroll
  for (int a = 5; a >= 0; --a) {   // R x = y
    double v = y[a];
#pragma unroll
    for (int m = a + 1; m < 6; ++m) v -= A[6 * a + m] * x[m];
    x[a] = v / A[7 * a];
  }
#pragma unroll
  for (int a = 0; a < 6; ++a)
    if (!isfinite(x[a])) return false;
  return true;
}

template <typename Real>
__global__ __launch_bounds__(64 * kPnpWaves) void k_pnp(PnpArgs A) {
  __shared__ double sCam[kMaxCams * 16];
  for (int k = threadIdx.x; k < A.n_cams * 16; k += blockDim.x) sCam[k] = A.cams[k];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int f = blockIdx.x * kPnpWaves + (threadIdx.x >> 6);
  if (f >= A.n_frames) return;   // whole wave
  const DevSettings S = A.settings;

  // structure checks on the device arrays: a frame that fails keeps its pose
  const long long o0 = A.frame_obs_begin[f], o1 = A.frame_obs_begin[f + 1];
  bool bad = !(0 <= o0 && o0 <= o1 && o1 <= A.n_obs);
  if (!bad) {
    bool b = false;
    for (long long o = o0 + lane; o < o1; o += 64) {
      const int p = A.obs_point[o];
      const int c = A.obs_cam ? A.obs_cam[o] : 0;
      b = b || p < 0 || p >= A.n_points || c < 0 || c >= A.n_cams;
    }
    bad = __any(b);
  }
  if (bad) {
    if (lane == 0 && A.reports) {
      ba_report r{};
      r.status = 2;
      A.reports[f] = r;
    }
    return;
  }

  double T[12], M[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) T[k] = A.poses[12 * (long long)f + k];
  const bool has_m = A.frame_transform != nullptr;
#pragma unroll
  for (int k = 0; k < 12; ++k) M[k] = has_m ? A.frame_transform[12 * (long long)f + k] : 0.0;

  // one pass over the frame's observations at pose P: the robust cost, and
  // (lin) U, g; (check) the depth test
  auto pass = [&](const double* P, bool lin, double* Ug, double& Fsum, bool& depth_bad) {
    Real U[21], g[6];
#pragma unroll
    for (int k = 0; k < 21; ++k) U[k] = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) g[k] = 0;
    double F = 0.0;
    bool dbad = false;
    for (long long o = o0 + lane; o < o1; o += 64) {
      const int c = A.obs_cam ? A.obs_cam[o] : 0;
      const double* C = sCam + 16 * c;
      double xb[3];
      frame_point(P, M, has_m, A.points + 3 * (long long)A.obs_point[o], xb);
      const double wo = A.obs_w ? A.obs_w[o] : 1.0;
      const double du = A.obs_uv[2 * o] - C[2], dv = A.obs_uv[2 * o + 1] - C[3];
      const Lin<Real> L = linearise<Real>(xb, C, du, dv, wo, S.huber_delta);
      dbad = dbad || !(L.Z > S.min_depth);
      F += L.rho_w;
      if (lin) {
        const Real w1 = (Real)(L.wo * L.d1);
        const Real* ar[2] = {L.a0, L.a1};
        Real J[2][6];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const Real* a = ar[k];
          J[k][0] = a[0];
          J[k][1] = a[1];
          J[k][2] = a[2];
          Real cr[3];
          cross3(L.xb, a, cr);
          J[k][3] = cr[0];
          J[k][4] = cr[1];
          J[k][5] = cr[2];
        }
        int e = 0;
#pragma unroll
        for (int r = 0; r < 6; ++r) {
          const Real wj0 = w1 * J[0][r], wj1 = w1 * J[1][r];
#pragma unroll
          for (int cc = r; cc < 6; ++cc, ++e) U[e] += wj0 * J[0][cc] + wj1 * J[1][cc];
          g[r] += wj0 * L.r[0] + wj1 * L.r[1];
        }
      }
    }
    Fsum = 0.5 * wave_total(F);
    depth_bad = __any(dbad);
    if (lin) {
#pragma unroll
      for (int k = 0; k < 21; ++k) Ug[k] = wave_total((double)U[k]);
#pragma unroll
      for (int k = 0; k < 6; ++k) Ug[21 + k] = wave_total((double)g[k]);
    }
  };

  double Ug[27];
  double F;
  bool dummy;
  pass(T, true, Ug, F, dummy);
  const double F0 = F;
  double lam = S.lambda_init;
  int acc = 0, chol = 0, depth = 0;
  for (int it = 0; it < S.max_iters; ++it) {
    ba_iter_trace tr;
    tr.cost = F;
    tr.lambda = lam;
    tr.cand_cost = __builtin_nan("");
    tr.status = 0;
    double d[6];
    bool accept = false;
    if (!solve6(Ug, Ug + 21, lam, d)) {
      tr.status = 1;
      ++chol;
    } else {
      double D[12], Tc[12];
      exp_se3(d, D);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b)
          Tc[4 * a + b] = D[4 * a] * T[b] + D[4 * a + 1] * T[4 + b] + D[4 * a + 2] * T[8 + b];
        Tc[4 * a + 3] = D[4 * a] * T[3] + D[4 * a + 1] * T[7] + D[4 * a + 2] * T[11] + D[4 * a + 3];
      }
      double Fc;
      bool dbad;
      pass(Tc, false, nullptr, Fc, dbad);
      if (dbad) {
        tr.status = 2;
        ++depth;
      } else {
        tr.cand_cost = Fc;
        accept = Fc < F;
      }
      if (accept) {
#pragma unroll
        for (int k = 0; k < 12; ++k) T[k] = Tc[k];
        F = Fc;
        ++acc;
        pass(T, true, Ug, Fc, dbad);   // U, g at the new pose (F stays the candidate's)
      }
    }
    lam = accept ? fmax(lam / S.lambda_down, S.lambda_min) : fmin(lam * S.lambda_up, S.lambda_max);
    tr.accepted = accept ? 1 : 0;
    if (lane == 0 && A.traces) A.traces[(long long)f * S.max_iters + it] = tr;
  }
  if (lane < 12) {
    double v = T[0];
#pragma unroll
    for (int k = 1; k < 12; ++k) v = lane == k ? T[k] : v;
    A.poses[12 * (long long)f + lane] = v;
  }
  if (lane == 0 && A.reports) {
    ba_report r;
    r.initial_cost = F0;
    r.final_cost = F;
    r.final_lambda = lam;
    r.iters = S.max_iters;
    r.accepted = acc;
    r.chol_failures = chol;
    r.depth_rejects = depth;
    r.status = isfinite(F0) ? 0 : 1;
    r.reserved = 0;
    A.reports[f] = r;
  }
}

template <typename Real>
hipError_t run_pnp(const PnpArgs& A) {
  if (A.n_frames <= 0) return hipSuccess;
  const int blocks = (A.n_frames + kPnpWaves - 1) / kPnpWaves;
  hipLaunchKernelGGL(k_pnp<Real>, dim3(blocks), dim3(64 * kPnpWaves), 0, (hipStream_t)A.stream, A);
  return hipGetLastError();
}

template hipError_t run_pnp<float>(const PnpArgs&);
template hipError_t run_pnp<double>(const PnpArgs&);

}  // namespace ba
