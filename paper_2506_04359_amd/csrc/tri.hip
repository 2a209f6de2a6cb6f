// gfx950 batched multi-view triangulation: every landmark re-estimated from its
// observations with the poses held fixed (paper Sec. 2.2, 3D module: new
// landmarks are triangulated from the multi-view observations of a keyframe
// before they enter the local map).
//
// One lane per landmark (a workgroup's landmarks ordered by observation count
// across its lanes); the landmark's observations are a contiguous range.  When
// the poses a workgroup reads span a range that, times the camera count, is at
// most 128, the world-to-camera transforms T_cb T_bw_i of that range are
// composed once into LDS, so each observation needs one transform and the
// Jacobian is A R_cw directly.
//   start     the weighted least-squares intersection of the viewing rays,
//             (sum w (I - d d^T)) p0 = sum w (I - d d^T) c, by a 3x3 FP64
//             Cholesky; fewer than two views or a pivot <= 1e-10 trace marks
//             the landmark degenerate (NaN point, status 3); a start at depth
//             <= min_depth in any view is returned unrefined (status 4)
//   refine    exactly max_iters LM attempts on the robust reprojection cost:
//             V = sum w rho' J^T J, g = sum w rho' J^T r (J the 2x3 point
//             Jacobian A R_c R_i, accumulated in Real), (V + lambda
//             diag(max(V_kk, 1e-9))) d = -g by FP64 Cholesky, candidate p + d,
//             depth guard, accept iff the FP64 cost strictly drops
// Each candidate's pass also forms V, g there, so an accepted attempt needs no
// second pass.  Lanes share nothing: no barrier, no atomics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.hpp"
#include "geometry.hpp"
#include "tri.hpp"

namespace ba {

constexpr int kTriThreads = 256;
constexpr int kTriPoseCache = 128;   // (pose, camera) transforms a workgroup keeps in LDS

// Cholesky solve of a 3x3 SPD system stored as (00, 01, 02, 11, 12, 22):
// x = A^-1 b.  False on a pivot <= floor or a non-finite one.
__device__ __forceinline__ bool solve3(const double* A, const double* b, double floor, double* x) {
  const double p0 = A[0];
  if (!(p0 > floor) || !isfinite(p0)) return false;
  const double i0 = rsqrt_nr(p0);
  const double l10 = A[1] * i0, l20 = A[2] * i0;
  const double p1 = A[3] - l10 * l10;
  if (!(p1 > floor) || !isfinite(p1)) return false;
  const double i1 = rsqrt_nr(p1);
  const double l21 = (A[4] - l20 * l10) * i1;
  const double p2 = A[5] - l20 * l20 - l21 * l21;
  if (!(p2 > floor) || !isfinite(p2)) return false;
  const double i2 = rsqrt_nr(p2);
  const double y0 = b[0] * i0;
  const double y1 = (b[1] - l10 * y0) * i1;
  const double y2 = (b[2] - l20 * y0 - l21 * y1) * i2;
  x[2] = y2 * i2;
  x[1] = (y1 - l21 * x[2]) * i1;
  x[0] = (y0 - l10 * x[1] - l20 * x[2]) * i0;
  return isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
}

// absent camera indices / weights read one constant entry (stride 0); global
// memory (not constant) keeps those loads global rather than flat
__device__ int kTriCamZero = 0;
__device__ double kTriWeightOne = 1.0;

// Ray start and LM refinement of landmark j (observations [o0, o1), indices
// already checked).  COMPOSED: P holds, per (pose i, camera c) at
// 16 ((i - pbase) n_cams + c), the camera record with the world-to-camera
// transform T_cb T_bw_i in place of T_cb (so the point goes to the camera in
// one transform and A R_cw is the Jacobian); otherwise P holds the poses
// (at 12 (i - pbase)) and the cameras come from sCam.
template <typename Real, bool COMPOSED>
__device__ __forceinline__ void tri_landmark(const TriArgs& A, int j, long long o0, long long o1,
                                             const double* sCam, const double* P, int pbase) {
  const DevSettings S = A.settings;
  const double kNaN = __builtin_nan("");
  const int* cp = A.obs_cam ? A.obs_cam : &kTriCamZero;
  const long long cstep = A.obs_cam ? 1 : 0;
  const double* wp = A.obs_w ? A.obs_w : &kTriWeightOne;
  const long long wstep = A.obs_w ? 1 : 0;
  auto finish = [&](int status, const double* p) {
    A.points[3 * (long long)j] = p ? p[0] : kNaN;
    A.points[3 * (long long)j + 1] = p ? p[1] : kNaN;
    A.points[3 * (long long)j + 2] = p ? p[2] : kNaN;
    if (A.reports) {
      ba_report r;
      r.initial_cost = kNaN;
      r.final_cost = kNaN;
      r.final_lambda = S.lambda_init;
      r.iters = 0;
      r.accepted = 0;
      r.chol_failures = 0;
      r.depth_rejects = 0;
      r.status = status;
      r.reserved = 0;
      A.reports[j] = r;
    }
  };
  if (o1 - o0 < 2) return finish(3, nullptr);

  // One observation: pose index, camera, pixel, weight.  The loops below load
  // observation o + 1 while observation o is computed.
  struct Ob {
    int i, c;
    double u, v, w;
  };
  auto load = [&](long long o) {
    Ob b;
    b.i = A.obs_pose[o];
    b.c = cp[o * cstep];
    b.u = A.obs_uv[2 * o];
    b.v = A.obs_uv[2 * o + 1];
    b.w = wp[o * wstep];
    return b;
  };

  // start: least-squares intersection of the viewing rays
  double M[6] = {0, 0, 0, 0, 0, 0}, mb[3] = {0, 0, 0};
  {
    Ob cur = load(o0);
    for (long long o = o0; o < o1; ++o) {
      const Ob nxt = load(o + 1 < o1 ? o + 1 : o);
      double Rcw[9], tcw[3];
      const double* C;
      if constexpr (COMPOSED) {
        C = P + 16 * ((cur.i - pbase) * A.n_cams + cur.c);
#pragma unroll
        for (int k = 0; k < 9; ++k) Rcw[k] = C[4 + k];
#pragma unroll
        for (int a = 0; a < 3; ++a) tcw[a] = C[13 + a];
      } else {
        const double* T = P + 12 * (cur.i - pbase);
        C = sCam + 16 * cur.c;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
          for (int b = 0; b < 3; ++b)
            Rcw[3 * a + b] = C[4 + 3 * a] * T[b] + C[5 + 3 * a] * T[4 + b] + C[6 + 3 * a] * T[8 + b];
          tcw[a] = C[4 + 3 * a] * T[3] + C[5 + 3 * a] * T[7] + C[6 + 3 * a] * T[11] + C[13 + a];
        }
      }
      const double v[3] = {(cur.u - C[2]) / C[0], (cur.v - C[3]) / C[1], 1.0};
      double d[3], ctr[3];
#pragma unroll
      for (int b = 0; b < 3; ++b) {   // world direction R_cw^T v and centre -R_cw^T t_cw
        d[b] = Rcw[b] * v[0] + Rcw[3 + b] * v[1] + Rcw[6 + b] * v[2];
        ctr[b] = -(Rcw[b] * tcw[0] + Rcw[3 + b] * tcw[1] + Rcw[6 + b] * tcw[2]);
      }
      const double in = rsqrt_nr(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      d[0] *= in;
      d[1] *= in;
      d[2] *= in;
      const double dc = d[0] * ctr[0] + d[1] * ctr[1] + d[2] * ctr[2];
      const double w = cur.w;
      M[0] += w * (1.0 - d[0] * d[0]);
      M[1] -= w * d[0] * d[1];
      M[2] -= w * d[0] * d[2];
      M[3] += w * (1.0 - d[1] * d[1]);
      M[4] -= w * d[1] * d[2];
      M[5] += w * (1.0 - d[2] * d[2]);
#pragma unroll
      for (int a = 0; a < 3; ++a) mb[a] += w * (ctr[a] - d[a] * dc);
      cur = nxt;
    }
  }
  double p[3];
  if (!solve3(M, mb, 1e-10 * (M[0] + M[3] + M[5]), p)) return finish(3, nullptr);

  // one pass at point q: the robust cost, the number of depths <= min_depth,
  // and V (00 01 02 11 12 22), g
  auto pass = [&](const double* q, double& F, int& nbad, Real* V, Real* g) {
#pragma unroll
    for (int k = 0; k < 6; ++k) V[k] = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) g[k] = 0;
    F = 0.0;
    nbad = 0;
    Ob cur = load(o0);
    for (long long o = o0; o < o1; ++o) {
      const Ob nxt = load(o + 1 < o1 ? o + 1 : o);
      Real J0[3], J1[3];
      Lin<Real> L;
      if constexpr (COMPOSED) {
        // the record's transform takes the world point to the camera: the
        // rows of A R_cw are the Jacobian
        const double* C = P + 16 * ((cur.i - pbase) * A.n_cams + cur.c);
        L = linearise<Real>(q, C, cur.u - C[2], cur.v - C[3], cur.w, S.huber_delta);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          J0[b] = L.a0[b];
          J1[b] = L.a1[b];
        }
      } else {
        const double* T = P + 12 * (cur.i - pbase);
        const double* C = sCam + 16 * cur.c;
        double xb[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) xb[a] = T[4 * a] * q[0] + T[4 * a + 1] * q[1] + T[4 * a + 2] * q[2] + T[4 * a + 3];
        L = linearise<Real>(xb, C, cur.u - C[2], cur.v - C[3], cur.w, S.huber_delta);
        // J rows = (rows of A R_c) R_i
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          J0[b] = L.a0[0] * (Real)T[b] + L.a0[1] * (Real)T[4 + b] + L.a0[2] * (Real)T[8 + b];
          J1[b] = L.a1[0] * (Real)T[b] + L.a1[1] * (Real)T[4 + b] + L.a1[2] * (Real)T[8 + b];
        }
      }
      nbad += (L.Z > S.min_depth) ? 0 : 1;
      F += L.rho_w;
      const Real w1 = (Real)(L.wo * L.d1);
      int e = 0;
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const Real wj0 = w1 * J0[r], wj1 = w1 * J1[r];
#pragma unroll
        for (int c = r; c < 3; ++c, ++e) V[e] = fma(wj1, J1[c], fma(wj0, J0[c], V[e]));
        g[r] = fma(wj1, L.r[1], fma(wj0, L.r[0], g[r]));
      }
      cur = nxt;
    }
    F *= 0.5;
  };

  Real V[6], g[3];
  double F;
  int nbad;
  pass(p, F, nbad, V, g);
  if (nbad > 0) return finish(4, p);
  const double F0 = F;
  double lam = S.lambda_init;
  int acc = 0, chol = 0, depth = 0;
  for (int it = 0; it < S.max_iters; ++it) {
    ba_iter_trace tr;
    tr.cost = F;
    tr.lambda = lam;
    tr.cand_cost = kNaN;
    tr.status = 0;
    double Ad[6] = {V[0], V[1], V[2], V[3], V[4], V[5]};
    const int dg[3] = {0, 3, 5};
#pragma unroll
    for (int k = 0; k < 3; ++k) Ad[dg[k]] += lam * fmax(Ad[dg[k]], 1e-9);
    const double mg[3] = {-(double)g[0], -(double)g[1], -(double)g[2]};
    double dlt[3];
    bool accept = false;
    if (!solve3(Ad, mg, 0.0, dlt)) {
      tr.status = 1;
      ++chol;
    } else {
      const double cand[3] = {p[0] + dlt[0], p[1] + dlt[1], p[2] + dlt[2]};
      Real Vc[6], gc[3];
      double Fc;
      int nb;
      pass(cand, Fc, nb, Vc, gc);
      if (nb > 0) {
        tr.status = 2;
        ++depth;
      } else {
        tr.cand_cost = Fc;
        accept = Fc < F;
      }
      if (accept) {
#pragma unroll
        for (int k = 0; k < 3; ++k) p[k] = cand[k];
#pragma unroll
        for (int k = 0; k < 6; ++k) V[k] = Vc[k];
#pragma unroll
        for (int k = 0; k < 3; ++k) g[k] = gc[k];
        F = Fc;
        ++acc;
      }
    }
    lam = accept ? fmax(lam / S.lambda_down, S.lambda_min) : fmin(lam * S.lambda_up, S.lambda_max);
    tr.accepted = accept ? 1 : 0;
    if (A.traces) A.traces[(long long)j * S.max_iters + it] = tr;
  }
  A.points[3 * (long long)j] = p[0];
  A.points[3 * (long long)j + 1] = p[1];
  A.points[3 * (long long)j + 2] = p[2];
  if (A.reports) {
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
    A.reports[j] = r;
  }
}

template <typename Real>
__global__ __launch_bounds__(kTriThreads) void k_tri(TriArgs A) {
  __shared__ double sCam[kMaxCams * 16];
  __shared__ double sComp[kTriPoseCache * 16];
  __shared__ int sCount[kTriThreads];
  __shared__ int sOrder[kTriThreads];
  __shared__ int sRange[2][kTriThreads / 64];
  for (int k = threadIdx.x; k < A.n_cams * 16; k += blockDim.x) sCam[k] = A.cams[k];
  // Lanes take the workgroup's landmarks in order of observation count (ties
  // by index), so that the lanes of a wave run loops of similar length.
  {
    const int jj = blockIdx.x * kTriThreads + threadIdx.x;
    long long n = 1ll << 30;   // past the end: sorted last
    if (jj < A.n_points) {
      n = (long long)A.point_obs_begin[jj + 1] - A.point_obs_begin[jj];
      n = n < 0 ? 0 : (n > (1ll << 29) ? (1ll << 29) : n);
    }
    sCount[threadIdx.x] = (int)n;
    __syncthreads();
    int rank = 0;
    for (int k = 0; k < kTriThreads; ++k) {
      const int c = sCount[k];
      rank += (c < (int)n || (c == (int)n && k < (int)threadIdx.x)) ? 1 : 0;
    }
    sOrder[rank] = threadIdx.x;
    __syncthreads();
  }
  const int j = blockIdx.x * kTriThreads + sOrder[threadIdx.x];

  // structure checks, and the range of pose indices the workgroup reads
  int status = 0, pmin = 0x7fffffff, pmax = -1;
  long long o0 = 0, o1 = 0;
  if (j < A.n_points) {
    o0 = A.point_obs_begin[j];
    o1 = A.point_obs_begin[j + 1];
    if (!(0 <= o0 && o0 <= o1 && o1 <= A.n_obs)) {
      status = 2;
    } else {
      for (long long o = o0; o < o1; ++o) {
        const int i = A.obs_pose[o], c = A.obs_cam ? A.obs_cam[o] : 0;
        if (i < 0 || i >= A.n_poses || c < 0 || c >= A.n_cams) status = 2;
        pmin = i < pmin ? i : pmin;
        pmax = i > pmax ? i : pmax;
      }
    }
    if (status) pmin = 0x7fffffff, pmax = -1;
  }
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const int a = __shfl_xor(pmin, m), b = __shfl_xor(pmax, m);
    pmin = a < pmin ? a : pmin;
    pmax = b > pmax ? b : pmax;
  }
  if ((threadIdx.x & 63) == 0) {
    sRange[0][threadIdx.x >> 6] = pmin;
    sRange[1][threadIdx.x >> 6] = pmax;
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kTriThreads / 64; ++w) {
    pmin = sRange[0][w] < pmin ? sRange[0][w] : pmin;
    pmax = sRange[1][w] > pmax ? sRange[1][w] : pmax;
  }
  // every index was checked against n_poses, so [pmin, pmax] is in range;
  // compose T_cb T_bw_i for every (pose, camera) the range holds
  const bool cached = pmax >= pmin && (long long)(pmax - pmin + 1) * A.n_cams <= kTriPoseCache;
  if (cached) {
    const int n = (pmax - pmin + 1) * A.n_cams;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
      const int i = pmin + r / A.n_cams, c = r % A.n_cams;
      const double* T = A.poses + 12 * (long long)i;
      const double* C = sCam + 16 * c;
      double* out = sComp + 16 * r;
      out[0] = C[0];
      out[1] = C[1];
      out[2] = C[2];
      out[3] = C[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b)
          out[4 + 3 * a + b] = C[4 + 3 * a] * T[b] + C[5 + 3 * a] * T[4 + b] + C[6 + 3 * a] * T[8 + b];
        out[13 + a] = C[4 + 3 * a] * T[3] + C[5 + 3 * a] * T[7] + C[6 + 3 * a] * T[11] + C[13 + a];
      }
    }
  }
  __syncthreads();
  if (j >= A.n_points) return;
  if (status) {
    const double kNaN = __builtin_nan("");
    A.points[3 * (long long)j] = kNaN;
    A.points[3 * (long long)j + 1] = kNaN;
    A.points[3 * (long long)j + 2] = kNaN;
    if (A.reports) {
      ba_report r;
      r.initial_cost = kNaN;
      r.final_cost = kNaN;
      r.final_lambda = A.settings.lambda_init;
      r.iters = 0;
      r.accepted = 0;
      r.chol_failures = 0;
      r.depth_rejects = 0;
      r.status = 2;
      r.reserved = 0;
      A.reports[j] = r;
    }
    return;
  }
  if (cached)
    tri_landmark<Real, true>(A, j, o0, o1, sCam, sComp, pmin);
  else
    tri_landmark<Real, false>(A, j, o0, o1, sCam, A.poses, 0);
}

template <typename Real>
hipError_t run_triangulate(const TriArgs& A) {
  if (A.n_points <= 0) return hipSuccess;
  const int blocks = (A.n_points + kTriThreads - 1) / kTriThreads;
  hipLaunchKernelGGL(k_tri<Real>, dim3(blocks), dim3(kTriThreads), 0, (hipStream_t)A.stream, A);
  return hipGetLastError();
}

template hipError_t run_triangulate<float>(const TriArgs&);
template hipError_t run_triangulate<double>(const TriArgs&);

}  // namespace ba
