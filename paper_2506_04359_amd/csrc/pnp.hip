// gfx950 motion-only bundle adjustment: many independent frames, each one pose
// refined against fixed landmarks (paper Sec. 2.2: stereo pose estimation,
// Eq. 4; the multi-camera rig, Eq. 6; the loop-closure relative pose against
// landmarks moved into a map frame by a known T^mw, Eq. 14).
//
// WPF waves (1, 2 or 4) per frame run every LM attempt of that frame inside
// one launch (the frames share nothing, so no grid-wide step is needed):
//   pass       lanes stride over the frame's observations at a pose: FP64
//              transform and residual, Huber weight, the robust cost, the
//              depth test, and the 2x6 pose Jacobian with U (21) and g (6)
//              accumulated per lane (FP32 in mixed mode); the 28 sums (and
//              the depth count) are reduce-scattered over the wave in FP64
//              (permlane swaps across rows, DPP mirrors within a row), then
//              added over the frame's waves through LDS in a fixed order
//   solve      every lane: (U + lambda diag(max(U_kk, 1e-9))) d = -g by a 6x6
//              FP64 Cholesky; a non-positive pivot rejects the attempt
//   candidate  T' = Exp(d) T (FP64) and one pass at T': any depth <=
//              min_depth rejects, else the robust cost decides
//   accept     F' < F (strict): T <- T', lambda / 10; else lambda x 10
// The candidate's pass also linearises at T', so an accepted attempt needs no
// second pass over the observations (a rejected one discards that U, g).
// Wave-uniform state lives in scalar registers or spread over lanes: lanes
// 2k and 2k+1 hold sum k (U, g, F, depth count), lane k < 12 holds T[k].
// Every wave of a frame takes the same decisions from the same sums.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "device.hpp"
#include "geometry.hpp"
#include "pnp.hpp"

namespace ba {

// threads per workgroup: four one-wave frames, or one frame of WPF waves (a
// workgroup never holds two frames that wait at barriers)
template <int WPF>
constexpr int pnp_threads() { return WPF == 1 ? 256 : 64 * WPF; }
constexpr int kPnpSums = 32;
__device__ int kCamZero = 0;          // global memory (not constant) keeps the loads
__device__ double kWeightOne = 1.0;   // below global loads rather than flat ones

// Exchange of 64-bit values between lane groups: rows 2-3 of a with rows 0-1
// of b (permlane32), odd rows of a with even rows of b (permlane16).
__device__ __forceinline__ void swap_rows32(double& a, double& b) {
  const long long ia = __double_as_longlong(a), ib = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ia, (unsigned)ib, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(ia >> 32), (unsigned)(ib >> 32), false, false);
  a = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
  b = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}
__device__ __forceinline__ void swap_rows16(double& a, double& b) {
  const long long ia = __double_as_longlong(a), ib = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ia, (unsigned)ib, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(ia >> 32), (unsigned)(ib >> 32), false, false);
  a = __longlong_as_double(((long long)hi[0] << 32) | lo[0]);
  b = __longlong_as_double(((long long)hi[1] << 32) | lo[1]);
}

// Reduce-scatter of 32 per-lane values over the wave: lanes 2k and 2k+1 end
// with the wave total of v[k].  Each step halves the list: the lanes on one
// side of a lane bit keep the first half, the others the second, and each
// adds its partner's copy of the half it keeps (bits 5 and 4 by permlane
// swaps, bits 3, 2, 1 by DPP row mirror, half-row mirror and quad xor 2).
__device__ __forceinline__ double wave_sums32(double (&v)[32], int lane) {
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    swap_rows32(v[i], v[16 + i]);
    v[i] += v[16 + i];
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    swap_rows16(v[i], v[8 + i]);
    v[i] += v[8 + i];
  }
  const bool b3 = lane & 8, b2 = lane & 4, b1 = lane & 2;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double keep = b3 ? v[4 + i] : v[i], send = b3 ? v[i] : v[4 + i];
    v[i] = keep + dpp_r<0x140, 0xf>(send);   // row_mirror
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const double keep = b2 ? v[2 + i] : v[i], send = b2 ? v[i] : v[2 + i];
    v[i] = keep + dpp_r<0x141, 0xf>(send);   // row_half_mirror
  }
  {
    const double keep = b1 ? v[1] : v[0], send = b1 ? v[0] : v[1];
    v[0] = keep + dpp_r<0x4e, 0xf>(send);    // quad_perm [2, 3, 0, 1]
  }
  return v[0] + dpp_r<0xb1, 0xf>(v[0]);      // quad_perm [1, 0, 3, 2]
}

// Value of a wave-uniform double in scalar registers.
__device__ __forceinline__ double uniform(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// v with lane K's value replaced by the wave-uniform x (lane k holds entry k
// of a lane-spread vector).
template <int K>
__device__ __forceinline__ double lane_set(double v, double x) {
  const long long b = __double_as_longlong(v), xb = __double_as_longlong(x);
  const int xlo = __builtin_amdgcn_readfirstlane((int)(xb & 0xffffffffll));
  const int xhi = __builtin_amdgcn_readfirstlane((int)(xb >> 32));
  int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  asm("v_writelane_b32 %0, %1, %2" : "+v"(lo) : "s"(xlo), "i"(K));
  asm("v_writelane_b32 %0, %1, %2" : "+v"(hi) : "s"(xhi), "i"(K));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// f(integral_constant<int, K>) for K = B .. E-1.
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

// C = A B for 3x4 [R | t] transforms (row-major).
__device__ __forceinline__ void compose(const double* A, const double* B, double* C) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int b = 0; b < 3; ++b)
      C[4 * a + b] = A[4 * a] * B[b] + A[4 * a + 1] * B[4 + b] + A[4 * a + 2] * B[8 + b];
    C[4 * a + 3] = A[4 * a] * B[3] + A[4 * a + 1] * B[7] + A[4 * a + 2] * B[11] + A[4 * a + 3];
  }
}

// Cholesky solve of the damped 6x6 system, in place on the packed upper
// triangle (row-major: entry (r, c), c >= r, at 6r - r(r-1)/2 + c - r): x =
// -(U + lam diag(max(U_kk, 1e-9)))^-1 g.  False on a non-positive or
// non-finite pivot.
__device__ __forceinline__ bool solve6(double* R /*21, overwritten*/, const double* g, double lam,
                                       double* x) {
  auto idx = [](int r, int c) { return 6 * r - r * (r - 1) / 2 + c - r; };
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double d = R[idx(k, k)];
    R[idx(k, k)] = d + lam * (d > 1e-9 ? d : 1e-9);
  }
  double ir[6];   // 1 / R_aa
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    double d = R[idx(a, a)];
#pragma unroll
    for (int m = 0; m < a; ++m) d -= R[idx(m, a)] * R[idx(m, a)];
    if (!(d > 0.0) || !isfinite(d)) return false;
    ir[a] = rsqrt_nr(d);
#pragma unroll
    for (int c = a + 1; c < 6; ++c) {
      double v = R[idx(a, c)];
#pragma unroll
      for (int m = 0; m < a; ++m) v -= R[idx(m, a)] * R[idx(m, c)];
      R[idx(a, c)] = v * ir[a];
    }
  }
  double y[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) {   // R^T y = -g
    double v = -g[a];
#pragma unroll
    for (int m = 0; m < a; ++m) v -= R[idx(m, a)] * y[m];
    y[a] = v * ir[a];
  }
#pragma unroll
  for (int a = 5; a >= 0; --a) {   // R x = y
    double v = y[a];
#pragma unroll
    for (int m = a + 1; m < 6; ++m) v -= R[idx(a, m)] * x[m];
    x[a] = v * ir[a];
  }
#pragma unroll
  for (int a = 0; a < 6; ++a)
    if (!isfinite(x[a])) return false;
  return true;
}

template <typename Real, int WPF>
__global__ __launch_bounds__(pnp_threads<WPF>()) void k_pnp(PnpArgs A) {
  constexpr int kFramesPerBlock = WPF == 1 ? 4 : 1;
  __shared__ double sCam[kMaxCams * 16];
  __shared__ double sSum[WPF > 1 ? 2 : 1][WPF][kPnpSums];   // per wave, two buffers
  for (int k = threadIdx.x; k < A.n_cams * 16; k += blockDim.x) sCam[k] = A.cams[k];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int sub = wave % WPF;   // the wave's part of its frame
  const int f = blockIdx.x * kFramesPerBlock + wave / WPF;
  // with several waves per frame the workgroup is that one frame: its waves
  // leave together and meet at every barrier below
  if (f >= A.n_frames) return;
  const DevSettings S = A.settings;

  // structure checks on the device arrays: a frame that fails keeps its pose
  const long long o0 = A.frame_obs_begin[f], o1 = A.frame_obs_begin[f + 1];
  bool bad = !(0 <= o0 && o0 <= o1 && o1 <= A.n_obs);
  if (!bad) {
    bool b = false;
    for (long long o = o0 + sub * 64 + lane; o < o1; o += 64 * WPF) {
      const int p = A.obs_point[o];
      const int c = A.obs_cam ? A.obs_cam[o] : 0;
      b = b || p < 0 || p >= A.n_points || c < 0 || c >= A.n_cams;
    }
    bad = WPF > 1 ? (__syncthreads_or(b) != 0) : __any(b);
  }
  if (bad) {
    if (sub == 0 && lane == 0 && A.reports) {
      ba_report r{};
      r.status = 2;
      A.reports[f] = r;
    }
    return;
  }

  const double* Mg = A.frame_transform ? A.frame_transform + 12 * (long long)f : nullptr;
  // absent camera indices / weights read one constant entry (stride 0)
  const int* cp = A.obs_cam ? A.obs_cam : &kCamZero;
  const long long cstep = A.obs_cam ? 1 : 0;
  const double* wp = A.obs_w ? A.obs_w : &kWeightOne;
  const long long wstep = A.obs_w ? 1 : 0;
  // lane k < 12 holds T[k]
  double t_lane = lane < 12 ? A.poses[12 * (long long)f + lane] : 0.0;
  int buf = 0;

  // One pass at the pose whose transform of the points is X (T, or T M with
  // the map-from-world M of Eq. 14): lanes 2k, 2k+1 of the result hold sum k
  // over the frame's observations (U packed upper, g, 2F, the number of
  // depths <= min_depth).
  auto pass = [&](const double* X) -> double {
    Real U[21], g[6];
#pragma unroll
    for (int k = 0; k < 21; ++k) U[k] = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) g[k] = 0;
    double Fl = 0.0, nbad = 0.0;
    // Software pipeline over the lane's observations o = base + lane + i *
    // stride: the landmark, pixel and weight of step i + 1 and the indices of
    // step i + 2 are in flight while step i is computed.  Lanes past the end
    // reload the frame's last observation and add nothing.
    const long long base = o0 + sub * 64, stride = 64 * WPF;
    const int n_it = base < o1 ? (int)((o1 - base + stride - 1) / stride) : 0;   // wave-uniform
    if (n_it > 0) {
      const long long last = o1 - 1;
      auto at = [&](int i) {
        const long long o = base + lane + (long long)i * stride;
        return o < o1 ? o : last;
      };
      struct Obs {
        double p[3], u, v, w;
        int c;
      };
      auto fetch = [&](long long o, int pi, int ci) {
        Obs b;
        const double* pp = A.points + 3 * (long long)pi;
        b.p[0] = pp[0];
        b.p[1] = pp[1];
        b.p[2] = pp[2];
        b.u = A.obs_uv[2 * o];
        b.v = A.obs_uv[2 * o + 1];
        b.w = wp[o * wstep];
        b.c = ci;
        return b;
      };
      long long oa = at(0), ob = at(1);
      int pi_b = A.obs_point[ob], ci_b = cp[ob * cstep];
      Obs cur = fetch(oa, A.obs_point[oa], cp[oa * cstep]);
      for (int i = 0; i < n_it; ++i) {
        const bool valid = base + lane + (long long)i * stride < o1;
        const long long oc = at(i + 2);
        const int pi_c = A.obs_point[oc], ci_c = cp[oc * cstep];
        const Obs nxt = fetch(ob, pi_b, ci_b);

        const double* C = sCam + 16 * cur.c;
        double xb[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
          xb[a] = X[4 * a] * cur.p[0] + X[4 * a + 1] * cur.p[1] + X[4 * a + 2] * cur.p[2] + X[4 * a + 3];
        const double wo = valid ? cur.w : 0.0;
        const Lin<Real> L = linearise<Real>(xb, C, cur.u - C[2], cur.v - C[3], wo, S.huber_delta);
        nbad += (valid && !(L.Z > S.min_depth)) ? 1.0 : 0.0;
        Fl += L.rho_w;
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
        for (int r = 0; r < 6; ++r) {   // two fused multiply-adds per entry
          const Real wj0 = w1 * J[0][r], wj1 = w1 * J[1][r];
#pragma unroll
          for (int cc = r; cc < 6; ++cc, ++e) U[e] = fma(wj1, J[1][cc], fma(wj0, J[0][cc], U[e]));
          g[r] = fma(wj1, L.r[1], fma(wj0, L.r[0], g[r]));
        }
        cur = nxt;
        ob = oc;
        pi_b = pi_c;
        ci_b = ci_c;
      }
    }
    double v[kPnpSums];
#pragma unroll
    for (int k = 0; k < 21; ++k) v[k] = (double)U[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) v[21 + k] = (double)g[k];
    v[27] = Fl;
    v[28] = nbad;
    v[29] = v[30] = v[31] = 0.0;
    double sum = wave_sums32(v, lane);
    if constexpr (WPF > 1) {
      // add the frame's waves in wave order; two buffers so that one barrier
      // per pass suffices
      if (!(lane & 1)) sSum[buf][sub][lane >> 1] = sum;
      __syncthreads();
      sum = sSum[buf][0][lane >> 1];
#pragma unroll
      for (int w = 1; w < WPF; ++w) sum += sSum[buf][w][lane >> 1];
      buf ^= 1;
    }
    return sum;
  };
  // the points' transform for the lane-spread pose tl: T, or T M
  auto point_transform = [&](double tl, double* X) {
    double T[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) T[k] = wave_bcast(tl, k);
    if (Mg) {
      double M[12], TM[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) M[k] = Mg[k];
      compose(T, M, TM);
#pragma unroll
      for (int k = 0; k < 12; ++k) X[k] = uniform(TM[k]);
    } else {
#pragma unroll
      for (int k = 0; k < 12; ++k) X[k] = T[k];
    }
  };

  double sums_cur;   // lane-spread sums at T
  {
    double X[12];
    point_transform(t_lane, X);
    sums_cur = pass(X);
  }
  double F = 0.5 * wave_bcast(sums_cur, 2 * 27);
  const double F0 = F;
  double lam = S.lambda_init;
  int acc = 0, chol = 0, depth = 0;
  for (int it = 0; it < S.max_iters; ++it) {
    ba_iter_trace tr;
    tr.cost = F;
    tr.lambda = lam;
    tr.cand_cost = __builtin_nan("");
    tr.status = 0;
    double Ug[27], d[6];
#pragma unroll
    for (int k = 0; k < 27; ++k) Ug[k] = wave_bcast(sums_cur, 2 * k);
    bool accept = false;
    if (!solve6(Ug, Ug + 21, lam, d)) {
      tr.status = 1;
      ++chol;
    } else {
      double D[12], T[12], Tc[12];
      exp_se3(d, D);
#pragma unroll
      for (int k = 0; k < 12; ++k) T[k] = wave_bcast(t_lane, k);
      compose(D, T, Tc);
      double tc_lane = 0.0;
      static_for<0, 12>([&](auto k) { tc_lane = lane_set<decltype(k)::value>(tc_lane, Tc[k]); });
      double X[12];
      point_transform(tc_lane, X);
      const double sums_new = pass(X);
      const double Fc = 0.5 * wave_bcast(sums_new, 2 * 27);
      if (wave_bcast(sums_new, 2 * 28) > 0.0) {
        tr.status = 2;
        ++depth;
      } else {
        tr.cand_cost = Fc;
        accept = Fc < F;
      }
      if (accept) {
        t_lane = tc_lane;
        sums_cur = sums_new;
        F = Fc;
        ++acc;
      }
    }
    lam = accept ? fmax(lam / S.lambda_down, S.lambda_min) : fmin(lam * S.lambda_up, S.lambda_max);
    tr.accepted = accept ? 1 : 0;
    if (sub == 0 && lane == 0 && A.traces) A.traces[(long long)f * S.max_iters + it] = tr;
  }
  if (sub == 0 && lane < 12) A.poses[12 * (long long)f + lane] = t_lane;
  if (sub == 0 && lane == 0 && A.reports) {
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

template <typename Real, int WPF>
static hipError_t launch_pnp(const PnpArgs& A) {
  constexpr int fpb = WPF == 1 ? 4 : 1;
  const int blocks = (A.n_frames + fpb - 1) / fpb;
  hipLaunchKernelGGL((k_pnp<Real, WPF>), dim3(blocks), dim3(pnp_threads<WPF>()), 0,
                     (hipStream_t)A.stream, A);
  return hipGetLastError();
}

int pnp_waves_per_frame(int n_frames, long long n_obs) {
  // enough waves to give every SIMD of the 256 CUs three, while each wave
  // keeps at least about four observations per lane per pass
  const long long avg = n_frames > 0 ? n_obs / n_frames : 0;
  int wpf = 1;
  while (wpf < 4 && (long long)n_frames * wpf < 3 * 1024 && avg >= 2 * wpf * 256) wpf *= 2;
  return wpf;
}

template <typename Real>
hipError_t run_pnp(const PnpArgs& A) {
  if (A.n_frames <= 0) return hipSuccess;
  switch (A.waves_per_frame) {
    case 1: return launch_pnp<Real, 1>(A);
    case 2: return launch_pnp<Real, 2>(A);
    case 4: return launch_pnp<Real, 4>(A);
    default: return hipErrorInvalidValue;
  }
}

template hipError_t run_pnp<float>(const PnpArgs&);
template hipError_t run_pnp<double>(const PnpArgs&);

}  // namespace ba
