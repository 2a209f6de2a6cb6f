// gfx950 kernels of the sliding-window sparse Levenberg-Marquardt bundle adjuster.
//
// The method (paper Sec. 2.2, Eq. 2 and Eq. 3, and the sentence after Eq. 3):
// per-observation pinhole reprojection residuals with a Huber kernel, the
// normal equations in blocks (U_i per pose, V_j per landmark, W_ij per
// pose-landmark pair), elimination of the landmarks by the Schur complement,
// a Cholesky solve of the reduced camera system for the poses, then point
// back-substitution.  One LM attempt is four launches over all windows of a
// batch:
//
//   pass_a     per chunk of landmarks: linearise every observation, reduce the
//              per-pair W, per-landmark V and per-pose U blocks, eliminate each
//              landmark (V* = L D L^T, Z = W L^-T |D|^-1/2) and accumulate the
//              chunk's private partial of S = U* - sum Z Z^T and of the reduced
//              right-hand side in LDS
//   sum        per window: the chunk partials added in FP64 in chunk order
//   reduce     per window: sum the chunk partials in FP64 in a fixed order,
//              damp, blocked Cholesky (6x6 blocks) of S, two triangular solves,
//              candidate poses T' = Exp(dp) T
//   pass_b     per chunk: re-linearise (cheaper than storing W), back-substitute
//              dl_j, candidate points, robust cost of the candidate
//   accept     per window: compare costs, update lambda, switch state buffers
//
// The observation stream is coalesced SoA (du, dv, w) in landmark-major order.
// Within a workgroup, a tile of at most TP pairs is handled one thread per pair
// (linearisation, the pair's own Schur term, DPP sums per pose), one thread per
// landmark (3x3 elimination) and one thread per (off-diagonal target block,
// three rows) for the Schur products listed by the plan (no atomics).
// Every kernel of the adjoint (ADJ = true) reuses the same passes with the exact
// Hessian, lambda = 0 and the loss cotangent as right-hand side.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.hpp"
#include "vi.hpp"
#include "geometry.hpp"

namespace ba {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ int xcd_chunk(int b, int G) {
  // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous run of chunks so that one window's chunks share an L2.
  const int q = G >> 3, r = G & 7;
  const int x = b & 7, k = b >> 3;
  return x * q + (x < r ? x : r) + k;
}


// Block accumulators of one pose-landmark pair.
template <typename Real>
struct PairAcc {
  Real U[21];   // upper triangle of the 6x6 pose block, row-major
  Real gp[6];   // pose gradient
  Real W[18];   // 6x3 pose-point block
  Real V[6];    // upper triangle of the 3x3 point block (00 01 02 11 12 22)
  Real gl[3];   // point gradient
};

template <typename Real>
__device__ __forceinline__ void pair_zero(PairAcc<Real>& A) {
#pragma unroll
  for (int k = 0; k < 21; ++k) A.U[k] = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) A.gp[k] = 0;
#pragma unroll
  for (int k = 0; k < 18; ++k) A.W[k] = 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) A.V[k] = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) A.gl[k] = 0;
}

// Add one observation: the Gauss-Newton blocks with IRLS weight w rho', and in
// ADJ mode the remaining terms of the exact Hessian (second derivatives of the
// residual and the rho'' term).
template <typename Real, bool ADJ>
__device__ __forceinline__ void pair_add(PairAcc<Real>& A, const Lin<Real>& L, const Real* Rp,
                                         bool free_pose, const double* C) {
  Real Jp[2][6], Jl[2][3];
  const Real* ar[2] = {L.a0, L.a1};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const Real* a = ar[k];
    Jp[k][0] = a[0];
    Jp[k][1] = a[1];
    Jp[k][2] = a[2];
    Real c[3];
    cross3(L.xb, a, c);
    Jp[k][3] = c[0];
    Jp[k][4] = c[1];
    Jp[k][5] = c[2];
#pragma unroll
    for (int m = 0; m < 3; ++m) Jl[k][m] = Rp[m] * a[0] + Rp[3 + m] * a[1] + Rp[6 + m] * a[2];
  }
  const Real w1 = (Real)(L.wo * L.d1);
  Real wJp[2][6], wJl[2][3];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
#pragma unroll
    for (int m = 0; m < 6; ++m) wJp[k][m] = w1 * Jp[k][m];
#pragma unroll
    for (int m = 0; m < 3; ++m) wJl[k][m] = w1 * Jl[k][m];
  }
  if (free_pose) {
    int u = 0;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
#pragma unroll
      for (int c = r; c < 6; ++c) A.U[u++] += wJp[0][r] * Jp[0][c] + wJp[1][r] * Jp[1][c];
      A.gp[r] += wJp[0][r] * L.r[0] + wJp[1][r] * L.r[1];
#pragma unroll
      for (int c = 0; c < 3; ++c) A.W[3 * r + c] += wJp[0][r] * Jl[0][c] + wJp[1][r] * Jl[1][c];
    }
  }
  {
    int v = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int c = r; c < 3; ++c) A.V[v++] += wJl[0][r] * Jl[0][c] + wJl[1][r] * Jl[1][c];
      A.gl[r] += wJl[0][r] * L.r[0] + wJl[1][r] * L.r[1];
    }
  }
  if constexpr (ADJ) {
    // 2 w rho'' (J^T r)(J^T r)^T
    Real q[9];
#pragma unroll
    for (int m = 0; m < 6; ++m) q[m] = Jp[0][m] * L.r[0] + Jp[1][m] * L.r[1];
#pragma unroll
    for (int m = 0; m < 3; ++m) q[6 + m] = Jl[0][m] * L.r[0] + Jl[1][m] * L.r[1];
    const Real w2 = (Real)(2.0 * L.wo * L.d2);
    // w rho' sum_k r_k Hess(r_k) = w rho' (B^T Q B + M(a)),  B = [I, -[x_b]x, R_i]
    const double X = L.X, Y = L.Y;
    const double iz = recip_nr(L.Z);
    const Real pxz = (Real)(-(double)L.r[0] * C[0] * iz * iz);
    const Real pyz = (Real)(-(double)L.r[1] * C[1] * iz * iz);
    const Real pzz = (Real)(2.0 * ((double)L.r[0] * C[0] * X + (double)L.r[1] * C[1] * Y) * iz * iz * iz);
    Real c0[3], c1[3], c2[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      c0[m] = (Real)C[4 + m];
      c1[m] = (Real)C[7 + m];
      c2[m] = (Real)C[10 + m];
    }
    Real Q[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        Q[a][b] = pxz * (c0[a] * c2[b] + c2[a] * c0[b]) + pyz * (c1[a] * c2[b] + c2[a] * c1[b]) +
                  pzz * c2[a] * c2[b];
    // columns of B
    Real Bc[9][3];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      Real e[3] = {0, 0, 0};
      e[m] = 1;
      Bc[m][0] = e[0];
      Bc[m][1] = e[1];
      Bc[m][2] = e[2];
      cross3(e, L.xb, Bc[3 + m]);   // e_m x x_b = -[x_b]x e_m
      Bc[6 + m][0] = Rp[0 + m];
      Bc[6 + m][1] = Rp[3 + m];
      Bc[6 + m][2] = Rp[6 + m];
    }
    Real QB[9][3];
#pragma unroll
    for (int n = 0; n < 9; ++n)
#pragma unroll
      for (int a = 0; a < 3; ++a)
        QB[n][a] = Q[a][0] * Bc[n][0] + Q[a][1] * Bc[n][1] + Q[a][2] * Bc[n][2];
    Real ab[3];
#pragma unroll
    for (int m = 0; m < 3; ++m) ab[m] = L.r[0] * L.a0[m] + L.r[1] * L.a1[m];
    const Real ax = ab[0] * L.xb[0] + ab[1] * L.xb[1] + ab[2] * L.xb[2];
    // M(a) entry (m, n) in (rho, phi, point) order
    auto Mab = [&](int m, int n) -> Real {
      if (m > n) {
        const int t = m;
        m = n;
        n = t;
      }
      if (m >= 3 && m < 6 && n >= 3 && n < 6) {
        const int a = m - 3, b = n - 3;
        return (Real)0.5 * (L.xb[a] * ab[b] + ab[a] * L.xb[b]) - (a == b ? ax : (Real)0);
      }
      if (m < 3 && n >= 3 && n < 6) {
        // M_rho,phi[a][b] = ([a]x)[a][b] / 2
        const int a = m, b = n - 3;
        Real sk;
        if (a == b) sk = 0;
        else if (a == 0) sk = (b == 1) ? -ab[2] : ab[1];
        else if (a == 1) sk = (b == 0) ? ab[2] : -ab[0];
        else sk = (b == 0) ? -ab[1] : ab[0];
        return (Real)0.5 * sk;
      }
      if (m >= 3 && m < 6 && n >= 6) {
        // M_phi,point = -[a]x R_i
        const int a = m - 3, c = n - 6;
        Real s[3];   // row a of [a]x
        if (a == 0) { s[0] = 0; s[1] = -ab[2]; s[2] = ab[1]; }
        else if (a == 1) { s[0] = ab[2]; s[1] = 0; s[2] = -ab[0]; }
        else { s[0] = -ab[1]; s[1] = ab[0]; s[2] = 0; }
        return -(s[0] * Rp[c] + s[1] * Rp[3 + c] + s[2] * Rp[6 + c]);
      }
      return (Real)0;
    };
    auto H2 = [&](int m, int n) -> Real {
      const Real t = Bc[m][0] * QB[n][0] + Bc[m][1] * QB[n][1] + Bc[m][2] * QB[n][2];
      return w1 * (t + Mab(m, n)) + w2 * q[m] * q[n];
    };
    if (free_pose) {
      int u = 0;
#pragma unroll
      for (int r = 0; r < 6; ++r) {
#pragma unroll
        for (int c = r; c < 6; ++c) A.U[u++] += H2(r, c);
#pragma unroll
        for (int c = 0; c < 3; ++c) A.W[3 * r + c] += H2(r, 6 + c);
      }
    }
    int v = 0;
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = r; c < 3; ++c) A.V[v++] += H2(6 + r, 6 + c);
  }
}

// 3x3 symmetric L D L^T (no pivoting).  V = (v00 v01 v02 v11 v12 v22).
// ok = all pivots positive (spd) or merely non-zero (indef).
template <typename Real>
struct LDL3 {
  Real l10, l20, l21;
  Real isd[3];   // |d_k|^-1/2
  Real sg[3];    // sign(d_k)
};

// Reciprocal and reciprocal square root: the hardware approximations in FP32
// (about 1 ulp; the FP32 blocks carry far larger rounding already), IEEE in
// FP64, whose results are compared with the oracle at 1e-9.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float rsqrt_r(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double rsqrt_r(double x) { return 1.0 / sqrt(x); }

template <typename Real>
__device__ __forceinline__ bool ldl3(const Real* V, bool spd, LDL3<Real>& F) {
  const Real d0 = V[0];
  const Real r0 = recip(d0);
  const Real l10 = V[1] * r0, l20 = V[2] * r0;
  const Real d1 = V[3] - l10 * l10 * d0;
  const Real l21 = (V[4] - l20 * l10 * d0) * recip(d1);
  const Real d2 = V[5] - l20 * l20 * d0 - l21 * l21 * d1;
  F.l10 = l10;
  F.l20 = l20;
  F.l21 = l21;
  const Real d[3] = {d0, d1, d2};
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const bool good = spd ? (d[k] > (Real)0) : (d[k] != (Real)0);
    ok = ok && good && isfinite((double)d[k]);
    const Real ad = fabs(d[k]);
    F.isd[k] = rsqrt_r(ad);
    F.sg[k] = d[k] < (Real)0 ? (Real)-1 : (Real)1;
  }
  return ok && isfinite((double)l10) && isfinite((double)l20) && isfinite((double)l21);
}

// solve L z = w (unit lower), then scale by |D|^-1/2: z_bar = |D|^-1/2 L^-1 w
template <typename Real>
__device__ __forceinline__ void ldl3_half(const LDL3<Real>& F, const Real* w, Real* z) {
  const Real z0 = w[0];
  const Real z1 = w[1] - F.l10 * z0;
  const Real z2 = w[2] - F.l20 * z0 - F.l21 * z1;
  z[0] = z0 * F.isd[0];
  z[1] = z1 * F.isd[1];
  z[2] = z2 * F.isd[2];
}

// x = V^-1 c = L^-T D^-1 L^-1 c
template <typename Real>
__device__ __forceinline__ void ldl3_solve(const LDL3<Real>& F, const Real* c, Real* x) {
  Real h[3];
  ldl3_half(F, c, h);
  const Real y0 = h[0] * F.isd[0] * F.sg[0];
  const Real y1 = h[1] * F.isd[1] * F.sg[1];
  const Real y2 = h[2] * F.isd[2] * F.sg[2];
  x[2] = y2;
  x[1] = y1 - F.l21 * x[2];
  x[0] = y0 - F.l10 * x[1] - F.l20 * x[2];
}

// V + lambda * diag(max(V_kk, 1e-9)) on the packed upper triangle
template <typename Real>
__device__ __forceinline__ void damp3(Real* V, double lam) {
  const int dI[3] = {0, 3, 5};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double v = (double)V[dI[k]];
    V[dI[k]] = (Real)(v + lam * (v > 1e-9 ? v : 1e-9));
  }
}

// Block-wide sum of a double, deterministic (fixed shuffle tree + fixed order).
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* scratch) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) scratch[wv] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < NT / 64; ++k) t += scratch[k];
  __syncthreads();
  return t;   // valid in thread 0
}

// Sum of v and maximum of m over the workgroup (both valid in thread 0);
// scratch holds 2 NT / 64 doubles.
template <int NT>
__device__ __forceinline__ double block_sum_max(double v, double& m, double* scratch) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    v += __shfl_down(v, off, 64);
    m = fmax(m, __shfl_down(m, off, 64));
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) {
    scratch[wv] = v;
    scratch[NT / 64 + wv] = m;
  }
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0) {
    for (int k = 0; k < NT / 64; ++k) t += scratch[k];
    m = scratch[NT / 64];
    for (int k = 1; k < NT / 64; ++k) m = fmax(m, scratch[NT / 64 + k]);
  }
  __syncthreads();
  return t;
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double* scratch) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) scratch[wv] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int k = 0; k < NT / 64; ++k) t = fmax(t, scratch[k]);
  __syncthreads();
  return t;   // valid in thread 0
}

// Exclusive scan of n (<= NT) ints in LDS, in place, total at a[n].
// Per-chunk flags and costs of a window's chunks [c0, c1), reduced by one
// wave: lane l takes chunks c0 + l, c0 + l + 64, ... in order (four loads in
// flight), then an xor butterfly adds the lanes.  The result used is lane 0's,
// whose order of additions is fixed, so the sum is the same on every run.
__device__ __forceinline__ void wave_chunk_sums(const int32_t* flag, const double* cost, int c0, int c1,
                                                bool need_cost, int lane, int& f_out, double& F_out) {
  int f = 0;
  double F = 0.0;
  for (int c = c0 + lane; c < c1; c += 4 * 64) {
    int fl[4];
    double cs[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int cc = c + 64 * b;
      const bool in = cc < c1;
      fl[b] = in ? flag[cc] : 0;
      cs[b] = in && need_cost ? cost[cc] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      f |= fl[b];
      F += cs[b];
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    f |= __shfl_xor(f, o, 64);
    F += __shfl_xor(F, o, 64);
  }
  f_out = __builtin_amdgcn_readfirstlane(f);
  F_out = wave_bcast(F, 0);
}

template <int NT>
__device__ __forceinline__ void block_scan(int* a, int n, int* scratch) {
  const int t = threadIdx.x;
  int v = t < n ? a[t] : 0;
  // inclusive scan inside the wave
  const int lane = t & 63, wv = t >> 6;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  if (lane == 63) scratch[wv] = v;
  __syncthreads();
  int base = 0;
  for (int k = 0; k < wv; ++k) base += scratch[k];
  int total = 0;
  for (int k = 0; k < NT / 64; ++k) total += scratch[k];
  const int orig = t < n ? a[t] : 0;
  __syncthreads();
  if (t < n) a[t] = base + v - orig;
  if (t == 0) a[n] = total;
  __syncthreads();
}

// ---------------------------------------------------------------------------
// LDS layout of the chunk kernels
// ---------------------------------------------------------------------------

struct ChunkLds {
  // window caches
  static constexpr int kPose = 64 * 12;   // doubles
  static constexpr int kCam = 32 * 16;    // doubles
};

// Window caches: poses (current state), camera table, free slots.
__device__ __forceinline__ void load_window(const DevPlan& P, const WinDev& W,
                                            const double* __restrict__ poses, double* sPose,
                                            double* sCam, int* sFree) {
  for (int k = threadIdx.x; k < W.n_poses * 12; k += blockDim.x) sPose[k] = poses[k];
  for (int k = threadIdx.x; k < W.n_cams * 16; k += blockDim.x)
    sCam[k] = P.cam[16 * W.cam_off + k];
  for (int k = threadIdx.x; k < W.n_poses; k += blockDim.x)
    sFree[k] = P.free_slot[W.pose_off + k];
}

// ---------------------------------------------------------------------------
// init, pack
// ---------------------------------------------------------------------------

template <typename Real>
__global__ void k_init(DevPlan P, DevWork<Real> K, DevSettings S) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= P.n_windows) return;
  WinState st;
  st.lambda = S.lambda_init;
  st.cost = 0.0;
  st.cand_cost = 0.0;
  st.init_cost = 0.0;
  st.cur = 0;
  st.fail = 0;
  st.accepted = st.chol_failures = st.depth_rejects = st.iters = st.status = st.frozen = 0;
  K.state[w] = st;
}

// Gather the user's observations (user order, FP64) into the plan-ordered SoA
// stream: du = u - cx, dv = v - cy (principal point removed before rounding to
// the stream precision), w.
template <typename Real>
__global__ void k_pack(DevPlan P, DevTiles T, DevWork<Real> K, DevUser U) {
  const int chunk = blockIdx.x;
  const int wi = T.chunk_window[chunk];
  const WinDev W = P.win[wi];
  const int t0 = T.chunk_tile_begin[chunk], t1 = T.chunk_tile_begin[chunk + 1];
  if (t1 <= t0) return;
  const int l0 = T.tile_lm_begin[t0], l1 = T.tile_lm_begin[t1];
  const int o0 = P.pair_obs_begin[P.lm_pair_begin[l0]];
  const int o1 = P.pair_obs_begin[P.lm_pair_begin[l1]];
  for (int o = o0 + threadIdx.x; o < o1; o += blockDim.x) {
    const int u = W.obs_off + P.obs_perm[o];
    const double* C = P.cam + 16 * (W.cam_off + P.obs_cam[o]);
    K.du[o] = (Real)(U.obs_uv[2 * u] - C[2]);
    K.dv[o] = (Real)(U.obs_uv[2 * u + 1] - C[3]);
    if (K.w) K.w[o] = (Real)U.obs_w[u];
  }
}

// ---------------------------------------------------------------------------
// pass A: linearise + per-landmark elimination + chunk partial of S
// ---------------------------------------------------------------------------

// One step of the segmented scan: v += (value of the source lane) where the
// source lane carries the same key.
template <typename Real, int N, int CTRL, int ROWMASK>
__device__ __forceinline__ void run_step(Real* v, int key) {
  const int k2 = dpp_i<CTRL, ROWMASK>(-2, key);
  const bool ok = k2 == key;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const Real t = dpp_r<CTRL, ROWMASK>(v[i]);
    if (ok) v[i] += t;
  }
}

// Inclusive prefix sums of v[0..N) over runs of lanes with equal key inside a
// wave (runs are contiguous: keys are sorted within the wave): after the call
// the last lane of each run holds the run's total.  DPP only (no LDS): four
// in-row shifts, then the two row broadcasts that carry a run across rows.
template <typename Real, int N>
__device__ __forceinline__ void run_sums(Real* v, int key) {
  run_step<Real, N, 0x111, 0xf>(v, key);   // row_shr:1
  run_step<Real, N, 0x112, 0xf>(v, key);   // row_shr:2
  run_step<Real, N, 0x114, 0xf>(v, key);   // row_shr:4
  run_step<Real, N, 0x118, 0xf>(v, key);   // row_shr:8
  run_step<Real, N, 0x142, 0xa>(v, key);   // row_bcast:15 into rows 1 and 3
  run_step<Real, N, 0x143, 0xc>(v, key);   // row_bcast:31 into rows 2 and 3
}

// Rows of one target block per Schur work unit in pass A (1, 2, 3 or 6): two
// rows read 8 Z rows per product for 36 FMAs and keep enough units per tile to
// balance the threads (measured faster than three or six rows per unit).
#ifndef BA_ROWS_PER_UNIT
#define BA_ROWS_PER_UNIT 2
#endif
constexpr int kRowsPerUnit = BA_ROWS_PER_UNIT;
static_assert(6 % kRowsPerUnit == 0, "rows per unit must divide 6");

// Per-pose sums of pass A: U - Z sigma Z^T (21, upper), reduced rhs (6), diag(U) (6).
constexpr int kPoseSums = 33;

// Upper-triangle entry e (0..20) of a 6x6 block -> row-major offset r*6+c.
constexpr int kUpperOffC[21] = {0, 1, 2, 3, 4, 5, 7, 8, 9, 10, 11, 14, 15, 16, 17,
                                21, 22, 23, 28, 29, 35};

// The same offset for a run-time e (no table: an indexed table in constant
// memory would cost a memory access): row r has 6 - r entries.
__device__ __forceinline__ int upper_off(int e) {
  const int r = (e >= 6) + (e >= 11) + (e >= 15) + (e >= 18) + (e >= 20);
  const int start = 6 * r - r * (r - 1) / 2;
  return 7 * r + (e - start);
}

// Adds component k of a pose's run sum into the partial: U - Z sigma Z^T
// (upper triangle of the diagonal block), reduced rhs, diag(U) (LM only).
template <typename Real, bool ADJ>
__device__ __forceinline__ void pose_sum_add1(Real* sS, Real* sB, Real* sD, int nf, int s, int k,
                                              Real x) {
  if (k < 21) {
    sS[kBS * blk_index(s, s, nf) + upper_off(k)] += x;
  } else if (k < 27) {
    sB[6 * s + (k - 21)] += x;
  } else if (!ADJ) {
    sD[6 * s + (k - 27)] += x;
  }
}

template <typename Real, bool ADJ>
__device__ __forceinline__ void pose_sums_add(Real* sS, Real* sB, Real* sD, int nf, int s,
                                              const Real* v) {
  Real* D = sS + kBS * blk_index(s, s, nf);
#pragma unroll
  for (int k = 0; k < 21; ++k) D[kUpperOffC[k]] += v[k];
#pragma unroll
  for (int k = 0; k < 6; ++k) sB[6 * s + k] += v[21 + k];
  if (!ADJ) {
#pragma unroll
    for (int k = 0; k < 6; ++k) sD[6 * s + k] += v[27 + k];
  }
}

// Stored row stride of a pair's Z_bar (6 rows of 3), unpadded: the Schur units
// are bound by LDS bandwidth, and a padded row (4 floats) carries a quarter of
// dead bytes; the 18-word pair stride also spreads pairs over more banks.
template <typename Real>
struct ZRow {
  static constexpr int R = 3;
  static constexpr int S = 6 * R;
};

// Words of a tile's product list kept in registers between its load (tile
// start) and its store to LDS (after phase 2).
template <int TP>
struct ListRegs {
  static constexpr int N = TP >= 256 ? 12 : 16;
};

// LDS carve of pass A.  The camera table, the window's poses (FP64, staged
// once per work item: a tile's pairs read them right at its start) and the
// reduced-system partial are sized by the launch's largest window; the
// per-tile buffers by TP (a tile holds at most TP / 2 landmarks).  The pair ->
// landmark map is kept only for the adjoint's Schur units.
template <typename Real, int TP>
struct PassALds {
  static constexpr int NW = TP / 64;
  static size_t bytes(int np, int nc, int nf, int list_bytes, bool adj) {
    const size_t nblk = (size_t)nf * (nf + 1) / 2;
    return (size_t)(nc * 16 + np * 12 + 16) * sizeof(double) + (64 + (adj ? TP : 0) + 4 + 8) * sizeof(int) +
           (nblk * kBS + 12 * (size_t)nf + (size_t)2 * NW * kPoseSums) * sizeof(Real) + 16 +
           ((size_t)TP * ZRow<Real>::S + (size_t)(TP / 2) * 12) * sizeof(Real) + 16 +
           ((size_t)list_bytes + 15) / 16 * 16;
  }
};

// FP32: at least two waves per SIMD (the register budget that LDS allows);
// FP64 runs one workgroup per CU anyway.
template <typename Real, int TP, bool ADJ>
__global__ __launch_bounds__(TP, (sizeof(Real) == 4 ? 2 : 1)) void k_pass_a(DevPlan P, DevTiles T, DevWork<Real> K,
                                               DevUser U, DevSettings S, int it, int cls_begin,
                                               LdsDims D) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int NW = TP / 64;
  constexpr int LR = ListRegs<TP>::N;
  constexpr int kZS = ZRow<Real>::S, ZR = ZRow<Real>::R;
  const int chunk = T.chunk_order[cls_begin + xcd_chunk(blockIdx.x, gridDim.x)];
  const int wi = T.chunk_window[chunk];
  const WinDev W = P.win[wi];
  const WinState& st = K.state[wi];
  if (!ADJ && st.frozen) return;   // the whole work item (every thread of it) returns
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cur = ADJ ? 0 : st.cur;
  const double lam = ADJ ? 0.0 : st.lambda;
  const double* poses = (cur ? K.poses_b : U.poses) + 12 * W.pose_off;
  const double* points = (cur ? K.points_b : U.points) + 3 * W.point_off;
  const int nf = W.n_free, nblk = nf * (nf + 1) / 2, nS = 6 * nf;

  double* sCam = reinterpret_cast<double*>(smem);             // nc * 16
  double* sPose = sCam + D.nc * 16;                           // np * 12
  double* sRed = sPose + D.np * 12;                           // 16
  int* sFree = reinterpret_cast<int*>(sRed + 16);             // 64
  int* sPL = sFree + 64;                                      // TP (adjoint): pair -> tile-local landmark
  int* sFlag = sPL + (ADJ ? TP : 0);                          // 4
  int* sBndSlot = sFlag + 4;                                  // 8: slot of each edge run (or -1)
  Real* sS = reinterpret_cast<Real*>(sBndSlot + 8);           // nblk * kBS
  Real* sB = sS + nblk * kBS;                                 // nS
  Real* sD = sB + nS;                                         // nS
  Real* sBnd = sD + nS;                                       // 2 * NW * kPoseSums: edge-run sums
  // 16-byte aligned carve by offsets from the LDS base (integer casts of the
  // pointers would lose the LDS address space and turn every access into a
  // flat one)
  const int oPZ = ((int)(reinterpret_cast<unsigned char*>(sBnd + 2 * NW * kPoseSums) - smem) + 15) & ~15;
  Real* sPZ = reinterpret_cast<Real*>(smem + oPZ);           // TP * kZS
  Real* sPV = sPZ;                                            // TP * 9: V, g (phases 1-2, before Z)
  Real* sLF = sPZ + TP * kZS;                                 // TP / 2 * 12: landmark factors
  const int oLst = ((int)(reinterpret_cast<unsigned char*>(sLF + (TP / 2) * 12) - smem) + 15) & ~15;
  uint32_t* sLst = reinterpret_cast<uint32_t*>(smem + oLst);  // product lists (stored in phase 1)

  const int4* trec = reinterpret_cast<const int4*>(T.tile_rec);
  const int4* prec = reinterpret_cast<const int4*>(T.pair_rec);
  const int t0 = T.chunk_tile_begin[chunk], t1 = T.chunk_tile_begin[chunk + 1];
  // The global data of a tile is fetched one tile ahead, in three steps:
  // tile records two tiles ahead, pair records one tile ahead (both issued
  // during tile t - 1), and the pairs' points and first observations at the
  // start of tile t - 1 (their pair records are there by then).
  int4 ta = make_int4(0, 0, 0, 0), tb = make_int4(0, 0, 0, 0), nta = ta, ntb = tb;
  int4 rec = make_int4(0, 0, 0, -1), nrec = rec;
  if (t0 < t1) {
    ta = trec[2 * t0];
    tb = trec[2 * t0 + 1];
    if (tid < ta.y) rec = prec[ta.x + tid];
  }
  if (t0 + 1 < t1) {
    nta = trec[2 * (t0 + 1)];
    ntb = trec[2 * (t0 + 1) + 1];
    if (tid < nta.y) nrec = prec[nta.x + tid];
  }

  for (int k = tid; k < W.n_cams * 16; k += TP) sCam[k] = P.cam[16 * W.cam_off + k];
  for (int k = tid; k < W.n_poses * 12; k += TP) sPose[k] = poses[k];
  for (int k = tid; k < W.n_poses; k += TP) sFree[k] = P.free_slot[W.pose_off + k];
  for (int k = tid; k < nblk * kBS + 2 * nS; k += TP) sS[k] = (Real)0;
  if (tid == 0) sFlag[0] = 0;
  __syncthreads();

  // a pair's point and first observation
  double px = 0, py = 0, pz = 0;
  Real du0 = 0, dv0 = 0, wo0 = 1;
  int cam0 = 0;
  // (threads without a pair read the window's first point and observation 0:
  // the loads are issued on every path, so the counter waits stay exact)
  auto fetch_pair = [&](const int4& r, bool on, double& x, double& y, double& z, Real& du, Real& dv, Real& wo,
                        int& cam) {
    const int o = on ? r.x : 0;
    const double* pt = points + 3 * (on ? r.y - W.point_off : 0);
    x = pt[0];
    y = pt[1];
    z = pt[2];
    cam = P.obs_cam[o];
    du = K.du[o];
    dv = K.dv[o];
    const Real wv = (K.w ? K.w : K.du)[o];   // a load on every path (the value is dropped without weights)
    wo = K.w ? wv : (Real)1;
  };
  if (t0 < t1) fetch_pair(rec, tid < ta.y, px, py, pz, du0, dv0, wo0, cam0);

  double cost = 0.0, gmax = 0.0;
  for (int t = t0; t < t1; ++t) {
    const int p0 = ta.x, nP = ta.y, l0 = ta.z, nL = ta.w;
    const int lw0 = tb.x, nseg = tb.y, nprod = tb.z;
    const int nwords = nseg + (nprod + 1) / 2;
    // this tile's pair: its pose (point and first observation are here
    // already), and the tile's list words
    const int q = (rec.z >> 8) & 255, pose = rec.z & 255, nobs = rec.z >> 16;
    const int slot = tid < nP ? rec.w : -1;
    const int o0 = rec.x, lm = rec.y;
    double Rt[12];
    if (tid < nP) {
      const double* pp = sPose + 12 * pose;
#pragma unroll
      for (int k = 0; k < 12; ++k) Rt[k] = pp[k];
    }
    // (unconditional, clamped to the tile's last landmark: loads issued on
    // every path keep the counter waits exact)
    const int lt = l0 + min(tid, nL > 0 ? nL - 1 : 0);
    const int lq0 = P.lm_pair_begin[lt] - p0, lq1 = P.lm_pair_begin[lt + 1] - p0;
    const bool lregs = nwords <= LR * TP;
    uint32_t lwv[LR];
    if (lregs) {
      // unconditional loads (clamped to the tile's last word; the table ends
      // with a padding word), so that waiting for them never waits for the
      // prefetches issued after them
      const int last = nwords > 0 ? nwords - 1 : 0;
#pragma unroll
      for (int k = 0; k < LR; ++k) lwv[k] = T.lists[lw0 + min(tid + k * TP, last)];
    }
    // In flight during this tile (issued after this tile's own loads: the
    // load counter retires in order, so waiting for the list words does not
    // wait for these): the tile record after the next one, and the next
    // tile's pairs' points and first observations.
    int4 nnta = nta, nntb = ntb;
    if (t + 2 < t1) {
      nnta = trec[2 * (t + 2)];
      nntb = trec[2 * (t + 2) + 1];
    }
    double npx = 0, npy = 0, npz = 0;
    Real ndu = 0, ndv = 0, nwo = 1;
    int ncam = 0;
    fetch_pair(nrec, t + 1 < t1 && tid < nta.y, npx, npy, npz, ndu, ndv, nwo, ncam);

    // ---- phase 1: thread t linearises its pair (free pairs sorted by slot)
    PairAcc<Real> A;
    pair_zero(A);
    if (tid < nP) {
      if (ADJ) sPL[q] = lm - l0;
      double xb[3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
        xb[a] = Rt[4 * a] * px + Rt[4 * a + 1] * py + Rt[4 * a + 2] * pz + Rt[4 * a + 3];
      Real Rp[9];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Rp[3 * a + b] = (Real)Rt[4 * a + b];
      {
        const double* C = sCam + 16 * cam0;
        const Lin<Real> L = linearise<Real>(xb, C, (double)du0, (double)dv0, (double)wo0, S.huber_delta);
        cost += L.rho_w;
        pair_add<Real, ADJ>(A, L, Rp, slot >= 0, C);
      }
      for (int o = o0 + 1; o < o0 + nobs; ++o) {
        const double* C = sCam + 16 * P.obs_cam[o];
        const double wo = K.w ? (double)K.w[o] : 1.0;
        const Lin<Real> L = linearise<Real>(xb, C, (double)K.du[o], (double)K.dv[o], wo,
                                            S.huber_delta);
        cost += L.rho_w;
        pair_add<Real, ADJ>(A, L, Rp, slot >= 0, C);
      }
#pragma unroll
      for (int k = 0; k < 6; ++k) sPV[9 * q + k] = A.V[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) sPV[9 * q + 6 + k] = A.gl[k];
    }
    // this tile's product lists (the previous tile's phase 4 has ended)
    if (lregs) {
#pragma unroll
      for (int k = 0; k < LR; ++k) {
        const int i = tid + k * TP;
        if (i < nwords) sLst[i] = lwv[k];
      }
    } else {
      for (int i = tid; i < nwords; i += TP) sLst[i] = T.lists[lw0 + i];
    }
    __syncthreads();

    // ---- phase 2: one thread per landmark: V*, L D L^T, h
    if (tid < nL) {
      const int lmg = l0 + tid;
      Real V[6] = {0, 0, 0, 0, 0, 0}, g[3] = {0, 0, 0};
      // the landmark's pairs summed in order; the next pair's values are read
      // while the current ones are added (at the end the last pair is read
      // again, not used)
      if (lq0 < lq1) {
        Real x[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) x[k] = sPV[9 * lq0 + k];
        for (int qq = lq0; qq < lq1; ++qq) {
          const int nq = qq + 1 < lq1 ? qq + 1 : qq;
          Real y[9];
#pragma unroll
          for (int k = 0; k < 9; ++k) y[k] = sPV[9 * nq + k];
#pragma unroll
          for (int k = 0; k < 6; ++k) V[k] += x[k];
#pragma unroll
          for (int k = 0; k < 3; ++k) g[k] += x[6 + k];
#pragma unroll
          for (int k = 0; k < 9; ++k) x[k] = y[k];
        }
      }
      Real c[3];
      if (!ADJ) {
        gmax = fmax(gmax, fmax(fabs((double)g[0]), fmax(fabs((double)g[1]), fabs((double)g[2]))));
        damp3(V, lam);
        c[0] = -g[0];
        c[1] = -g[1];
        c[2] = -g[2];
      } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) c[k] = U.grad_points ? (Real)U.grad_points[3 * lmg + k] : (Real)0;
      }
      LDL3<Real> F;
      if (!ldl3(V, !ADJ, F)) sFlag[0] = 1;
      Real hb[3];
      ldl3_half(F, c, hb);
      Real* f = sLF + 12 * tid;
      f[0] = F.l10;
      f[1] = F.l20;
      f[2] = F.l21;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        f[3 + k] = F.isd[k];
        f[6 + k] = F.sg[k];
        f[9 + k] = hb[k];
      }
    }
    __syncthreads();
    // the pair records of the tile after the next one (its tile record has
    // arrived by now)
    // (unconditional, clamped: the values of threads without a pair are not used)
    const int4 nnrec = prec[nnta.x + min(tid, nnta.y > 0 ? nnta.y - 1 : 0)];

    // ---- phase 3: Z_bar = W L^-T |D|^-1/2 of this pair, its reduced rhs and
    // its own diagonal Schur term U - Z_bar sigma Z_bar^T (the products of a
    // pair with itself never enter the product lists), plus diag(U) for the
    // damping; then per-pose sums over adjacent lanes, added once per run
    Real v[kPoseSums];
    if (slot >= 0) {
      const Real* f = sLF + 12 * (lm - l0);
      LDL3<Real> F;
      F.l10 = f[0];
      F.l20 = f[1];
      F.l21 = f[2];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        F.isd[k] = f[3 + k];
        F.sg[k] = f[6 + k];
      }
      Real sh[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) sh[k] = f[6 + k] * f[9 + k];
      Real* Z = sPZ + kZS * q;
      Real z[6][3];
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        ldl3_half(F, A.W + 3 * r, z[r]);
        Z[ZR * r] = z[r][0];
        Z[ZR * r + 1] = z[r][1];
        Z[ZR * r + 2] = z[r][2];
        if (ZR == 4) Z[ZR * r + 3] = (Real)0;
        v[21 + r] = (ADJ ? (Real)0 : -A.gp[r]) - (z[r][0] * sh[0] + z[r][1] * sh[1] + z[r][2] * sh[2]);
      }
      int e = 0;
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        const Real zs0 = z[r][0] * F.sg[0], zs1 = z[r][1] * F.sg[1], zs2 = z[r][2] * F.sg[2];
        v[27 + r] = A.U[e];   // diagonal entry (r, r)
#pragma unroll
        for (int c = r; c < 6; ++c, ++e)
          v[e] = A.U[e] - (zs0 * z[c][0] + zs1 * z[c][1] + zs2 * z[c][2]);
      }
    } else {
#pragma unroll
      for (int k = 0; k < kPoseSums; ++k) v[k] = (Real)0;
    }
    run_sums<Real, kPoseSums>(v, slot);
    {
      // The last lane of each run holds the run's sum.  A run inside the wave
      // is the only one of its pose in the tile (pairs are ordered by pose):
      // it adds into the partial directly.  The runs holding lane 0 or lane 63
      // may continue in the neighbouring waves: they go to this wave's two
      // edge slots, folded in phase 4.
      const int next = __shfl_down(slot, 1, 64);
      const int slot0 = __builtin_amdgcn_readlane(slot, 0);
      const int slot63 = __builtin_amdgcn_readlane(slot, 63);
      const bool tail = slot >= 0 && (lane == 63 || next != slot);
      if (lane == 0) {
        sBndSlot[2 * wave] = slot0 >= 0 ? slot0 : -1;
        sBndSlot[2 * wave + 1] = (slot63 >= 0 && slot63 != slot0) ? slot63 : -1;
      }
      if (tail) {
        if (slot == slot0 || lane == 63) {
          Real* dst = sBnd + (2 * wave + (slot == slot0 ? 0 : 1)) * kPoseSums;
#pragma unroll
          for (int k = 0; k < kPoseSums; ++k) dst[k] = v[k];
        } else {
          pose_sums_add<Real, ADJ>(sS, sB, sD, nf, slot, v);
        }
      }
    }
    __syncthreads();
    // edge runs of the waves, one thread per component (the targets are
    // diagonal blocks, rhs and diag(U); phase 4 below writes only
    // off-diagonal blocks).  The last wave does it: it gets the shortest Schur
    // units of every round.  A run spanning waves leaves its pieces in
    // consecutive edge slots: they are summed in wave order in registers and
    // added to the partial once.
    if (tid >= TP - kPoseSums) {
      const int k = tid - (TP - kPoseSums);
      int sl[2 * NW];
      Real x[2 * NW];
#pragma unroll
      for (int b = 0; b < 2 * NW; ++b) {
        sl[b] = sBndSlot[b];
        x[b] = sBnd[b * kPoseSums + k];
      }
      int cur = -1;
      Real acc = (Real)0;
#pragma unroll
      for (int b = 0; b < 2 * NW; ++b) {
        if (sl[b] < 0) continue;
        if (sl[b] == cur) {
          acc += x[b];
        } else {
          if (cur >= 0) pose_sum_add1<Real, ADJ>(sS, sB, sD, nf, cur, k, acc);
          cur = sl[b];
          acc = x[b];
        }
      }
      if (cur >= 0) pose_sum_add1<Real, ADJ>(sS, sB, sD, nf, cur, k, acc);
    }

    // ---- phase 4: Schur blocks.  Unit (segment, rows r0..r0+kRowsPerUnit-1)
    // owns those rows of one off-diagonal target block for this tile: it sums
    // -Z_a[r] sigma Z_c^T over the segment's products in registers and
    // updates its rows of the partial once.
    const uint16_t* sProd = reinterpret_cast<const uint16_t*>(sLst + nseg);
    {
      constexpr int RG = kRowsPerUnit, UPS = 6 / RG;
      const int nun = nseg * UPS;
      for (int u = tid; u < nun; u += TP) {
        const uint32_t wd = sLst[u / UPS];
        const int r0 = (u % UPS) * RG;
        const int blk = wd & 1023, start = (wd >> 10) & 8191, len = wd >> 23;
        Real acc[RG][6];
#pragma unroll
        for (int i = 0; i < RG; ++i)
#pragma unroll
          for (int c = 0; c < 6; ++c) acc[i][c] = (Real)0;
        // Two register sets in turn: the Z rows of the next product (and the
        // index of the one after) are read while the current product is
        // multiplied, so a unit waits for LDS once per product.  At a unit's
        // end the reads are clamped to its last product (read, not used).
        Real a0[RG][3], z0[6][3], a1[RG][3], z1[6][3];
        auto load_rows = [&](uint32_t pp, Real (&a)[RG][3], Real (&z)[6][3]) {
          const int qa = pp & 255, qc = pp >> 8;
          const Real* Za = sPZ + kZS * qa + ZR * r0;
          const Real* Zc = sPZ + kZS * qc;
#pragma unroll
          for (int i = 0; i < RG; ++i)
#pragma unroll
            for (int m = 0; m < 3; ++m) a[i][m] = Za[ZR * i + m];
#pragma unroll
          for (int c = 0; c < 6; ++c)
#pragma unroll
            for (int m = 0; m < 3; ++m) z[c][m] = Zc[ZR * c + m];
          if (ADJ) {
            const Real* g = sLF + 12 * sPL[qa] + 6;
#pragma unroll
            for (int i = 0; i < RG; ++i)
#pragma unroll
              for (int m = 0; m < 3; ++m) a[i][m] *= g[m];
          }
        };
        // acc += a z^T as a chain of FMAs (one rounding per term)
        auto madd = [&](const Real (&a)[RG][3], const Real (&z)[6][3]) {
#pragma unroll
          for (int i = 0; i < RG; ++i)
#pragma unroll
            for (int c = 0; c < 6; ++c) {
              acc[i][c] = fma(a[i][0], z[c][0], acc[i][c]);
              acc[i][c] = fma(a[i][1], z[c][1], acc[i][c]);
              acc[i][c] = fma(a[i][2], z[c][2], acc[i][c]);
            }
        };
        const int end = start + len, last = end - 1;
        if (len > 0) {
          uint32_t i1 = sProd[min(start + 1, last)];
          load_rows(sProd[start], a0, z0);
          for (int k = start;; k += 2) {
            const uint32_t i2 = sProd[min(k + 2, last)];
            load_rows(i1, a1, z1);
            madd(a0, z0);
            if (k + 1 >= end) break;
            const uint32_t i3 = sProd[min(k + 3, last)];
            load_rows(i2, a0, z0);
            madd(a1, z1);
            if (k + 2 >= end) break;
            i1 = i3;
          }
        }
        Real* B = sS + kBS * blk + 6 * r0;
#pragma unroll
        for (int i = 0; i < RG; ++i)
#pragma unroll
          for (int c = 0; c < 6; ++c) B[6 * i + c] -= acc[i][c];
      }
    }
    __syncthreads();
    ta = nta;
    tb = ntb;
    nta = nnta;
    ntb = nntb;
    rec = nrec;
    nrec = nnrec;
    px = npx;
    py = npy;
    pz = npz;
    du0 = ndu;
    dv0 = ndv;
    wo0 = nwo;
    cam0 = ncam;
  }

  // ---- chunk partial out (the last tile's phase 4 ended with a barrier)
  Real* part = K.part + T.chunk_part_off[chunk];
  for (int k = tid; k < nblk * kBS + 2 * nS; k += TP) part[k] = sS[k];
  // the cost sum and the landmark-gradient maximum in one reduction
  double gm = gmax;
  const double tot = block_sum_max<TP>(cost, gm, sRed);
  if (tid == 0) {
    K.part_cost_a[chunk] = tot;
    K.part_flag_a[chunk] = sFlag[0];
    if (!ADJ) K.part_gmax[chunk] = gm;
  }
}

// ---------------------------------------------------------------------------
// reduce + blocked Cholesky of S + candidate poses (one workgroup per window)
// ---------------------------------------------------------------------------


// LDS stride of a 6x6 block in the reduction workgroup: dense, so every row
// pair of a block starts 16 bytes aligned and is read with one 128-bit LDS
// read (the chunk partials keep the odd stride kBS, which spreads the banks of
// the accumulating workgroups).
constexpr int kRS = 36;

// Waits for the LDS reads that produced v before anything that uses v: the
// reads of a step are issued together and waited for once, instead of the
// compiler's interleaving of each read with its first use.
template <int N>
__device__ __forceinline__ void lds_fence(double (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) __asm__ volatile("" : "+v"(v[i]));
}

// Upper Cholesky of one symmetric 6x6 block, by one wave: lane l < 36 brings
// entry (l / 6, l % 6).  Writes the upper triangle of R to D and 1 / R_pp to
// inv; raises *fail on a non-positive or non-finite pivot.  The lanes put
// their entries into D, then every lane factors the whole block in registers
// (the same values in every lane): the serial pivot chain has no cross-lane
// traffic.
__device__ __forceinline__ void factor_diag(double a, double* D, double* inv, int* fail) {
  const int lane = threadIdx.x & 63;
  if (lane < 36) D[lane] = a;
  __builtin_amdgcn_wave_barrier();
  double R[21];   // upper triangle, row-major: row p starts at 6 p - p (p - 1) / 2
#pragma unroll
  for (int p = 0, e = 0; p < 6; ++p)
#pragma unroll
    for (int q = p; q < 6; ++q, ++e) R[e] = D[6 * p + q];
  lds_fence(R);
  __builtin_amdgcn_wave_barrier();
  double ir6[6];
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    const int rp = 6 * p - p * (p - 1) / 2;   // (p, p)
    const double d = R[rp];
    if (!(d > 0.0) || !isfinite(d)) {   // the same in every lane
      if (lane == 0) *fail = 1;
      return;
    }
    const double ir = rsqrt(d), sd = d * ir;
    ir6[p] = ir;
    R[rp] = sd;
#pragma unroll
    for (int q = p + 1; q < 6; ++q) R[rp + q - p] *= ir;
#pragma unroll
    for (int x = p + 1; x < 6; ++x) {
      const int rx = 6 * x - x * (x - 1) / 2;
#pragma unroll
      for (int q = x; q < 6; ++q) R[rx + q - x] -= R[rp + x - p] * R[rp + q - p];
    }
  }
  // every lane holds the same factor: lane 0 stores it (27 stores instead of
  // a per-lane selection of its entry)
  if (lane == 0) {
#pragma unroll
    for (int p = 0, e = 0; p < 6; ++p)
#pragma unroll
      for (int q = p; q < 6; ++q, ++e) D[6 * p + q] = R[e];
#pragma unroll
    for (int p = 0; p < 6; ++p) inv[p] = ir6[p];
  }
}

// One item of the trailing update of step k of the blocked Cholesky in the
// reduction workgroup: RG rows of one block of the upper pairs k < i <= j
// (S_ij -= R_ki^T R_kj; the next diagonal block is excluded), or, past the
// npair blocks, of the right-hand side (b_i -= R_ki^T y_k).  A block splits
// into 6 / RG items: rows 4s, 4s + 1, 2 + s for RG = 3, rows 2s, 2s + 1 for
// RG = 2, row s for RG = 1, so a row pair is one 128-bit read.  Every read is
// issued before the first product; each entry is summed over m in order and
// then subtracted, whatever RG.
template <int RG>
__device__ __forceinline__ void trail_item(double* sS, double* sB, int k, int nf, int nt, int npair, int e) {
  constexpr int G = 6 / RG;
  const int sub = e % G, blkno = e / G;
  int rows[3];
  if (RG == 3) {
    rows[0] = 4 * sub;
    rows[1] = 4 * sub + 1;
    rows[2] = 2 + sub;
  } else if (RG == 2) {
    rows[0] = 2 * sub;
    rows[1] = 2 * sub + 1;
    rows[2] = 0;
  } else {
    rows[0] = sub;
    rows[1] = rows[2] = 0;
  }
  const bool rhs = blkno >= npair;
  int i, j = 0;
  if (rhs) i = blkno - npair;
  else upper_pair(blkno + 1, nt, i, j);
  const double* A = sS + kRS * blk_index(k, k + 1 + i, nf);
  double u[6][RG];
#pragma unroll
  for (int m = 0; m < 6; ++m) {
    if (RG >= 2) {
      const double2 a01 = *reinterpret_cast<const double2*>(A + 6 * m + rows[0]);
      u[m][0] = a01.x;
      u[m][1] = a01.y;
      if (RG == 3) u[m][RG - 1] = A[6 * m + rows[2]];
    } else {
      u[m][0] = A[6 * m + rows[0]];
    }
  }
  if (!rhs) {
    const double* Bm = sS + kRS * blk_index(k, k + 1 + j, nf);
    double* D = sS + kRS * blk_index(k + 1 + i, k + 1 + j, nf);
    double v[6][6], d[RG][6];
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
      for (int c = 0; c < 6; c += 2) {
        const double2 b2 = *reinterpret_cast<const double2*>(Bm + 6 * m + c);
        v[m][c] = b2.x;
        v[m][c + 1] = b2.y;
      }
#pragma unroll
    for (int r = 0; r < RG; ++r)
#pragma unroll
      for (int c = 0; c < 6; c += 2) {
        const double2 d2 = *reinterpret_cast<const double2*>(D + 6 * rows[r] + c);
        d[r][c] = d2.x;
        d[r][c + 1] = d2.y;
      }
    double acc[RG][6];
#pragma unroll
    for (int r = 0; r < RG; ++r)
#pragma unroll
      for (int c = 0; c < 6; ++c) acc[r][c] = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m)
#pragma unroll
      for (int r = 0; r < RG; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[r][c] += u[m][r] * v[m][c];
#pragma unroll
    for (int r = 0; r < RG; ++r)
#pragma unroll
      for (int c = 0; c < 6; c += 2)
        *reinterpret_cast<double2*>(D + 6 * rows[r] + c) =
            make_double2(d[r][c] - acc[r][c], d[r][c + 1] - acc[r][c + 1]);
  } else {
    double yk[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) yk[m] = sB[6 * k + m];
    double* bi = sB + 6 * (k + 1 + i);
#pragma unroll
    for (int r = 0; r < RG; ++r) {
      double v = 0.0;
#pragma unroll
      for (int m = 0; m < 6; ++m) v += u[m][r] * yk[m];
      bi[rows[r]] -= v;
    }
  }
}

// Sum of a window's chunk partials in FP64 (grid: windows x slices).  The
// workgroup's 256 threads form G = W.sum_groups groups of 256 / G entry
// lanes; each thread keeps kSumE entries of its slice, group g adds chunks
// g, g + G, ... (four in flight per step) and the groups' sums are added in
// group order through LDS.  The partials of a window are contiguous, one
// per chunk, so the chunk addresses need no table lookup.
template <typename Real>
__global__ __launch_bounds__(256) void k_sum(DevPlan P, DevTiles T, DevWork<Real> K, int wbase) {
  __shared__ double sG[kSumE][256];
  const int wi = T.win_order[wbase + blockIdx.x];
  if (K.state[wi].frozen) return;
  const WinDev W = P.win[wi];
  const int nf = W.n_free, nblk = nf * (nf + 1) / 2;
  const int ne = nblk * kBS + 12 * nf;
  const int G = W.sum_groups, L = 256 / G;
  const int g = threadIdx.x / L, l = threadIdx.x - g * L;
  const int e0 = blockIdx.y * (L * kSumE);
  if (e0 >= ne) return;
  const int nch = W.chunk_end - W.chunk_begin;
  const Real* base = K.part + (nch > 0 ? T.chunk_part_off[W.chunk_begin] : 0);
  // loads are unconditional (entries past the end read the last entry and
  // are dropped), so a step's 16 loads are all in flight before the first
  // is waited for
  int ec[kSumE];
  bool in[kSumE];
#pragma unroll
  for (int k = 0; k < kSumE; ++k) {
    const int e = e0 + l + L * k;
    in[k] = e < ne;
    ec[k] = in[k] ? e : ne - 1;
  }
  double acc[kSumE];
#pragma unroll
  for (int k = 0; k < kSumE; ++k) acc[k] = 0.0;
  int c = g;
  for (; c + 3 * G < nch; c += 4 * G) {
    Real v[4][kSumE];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const Real* a = base + (int64_t)(c + j * G) * ne;
#pragma unroll
      for (int k = 0; k < kSumE; ++k) v[j][k] = a[ec[k]];
    }
#pragma unroll
    for (int k = 0; k < kSumE; ++k)
      acc[k] += (((double)v[0][k] + (double)v[1][k]) + (double)v[2][k]) + (double)v[3][k];
  }
  for (; c < nch; c += G) {
    const Real* a = base + (int64_t)c * ne;
#pragma unroll
    for (int k = 0; k < kSumE; ++k) acc[k] += (double)a[ec[k]];
  }
  double* dst = K.ssum + W.sum_off;
  if (G == 1) {
#pragma unroll
    for (int k = 0; k < kSumE; ++k)
      if (in[k]) dst[ec[k]] = acc[k];
    return;
  }
#pragma unroll
  for (int k = 0; k < kSumE; ++k) sG[k][threadIdx.x] = acc[k];
  __syncthreads();
  if (g == 0) {
#pragma unroll
    for (int k = 0; k < kSumE; ++k) {
      double t = sG[k][l];
      for (int h = 1; h < G; ++h) t += sG[k][h * L + l];
      if (in[k]) dst[ec[k]] = t;
    }
  }
}

template <typename Real, int NT, bool ADJ>
__global__ __launch_bounds__(NT) void k_reduce(DevPlan P, DevTiles T, DevWork<Real> K, DevUser U,
                                               DevSettings S, int it, int wbase) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wi = T.win_order[wbase + blockIdx.x];
  const WinDev W = P.win[wi];
  WinState& st = K.state[wi];
  const int tid = threadIdx.x;
  const int nf = W.n_free, nblk = nf * (nf + 1) / 2, nS = 6 * nf;
  double* sS = reinterpret_cast<double*>(smem);   // nblk * kRS
  double* sB = sS + nblk * kRS;                   // nS
  double* sD = sB + nS;                           // nS
  double* sInv = sD + nS;                         // nS: 1 / R_pp of the diagonal blocks
  int* sFail = reinterpret_cast<int*>(sInv + nS); // 2 ints (one double): failure, freeze
  double* sMax = sInv + nS + 1;                   // NT / 64 (<= 8): freeze test
  const int c0 = W.chunk_begin, c1 = W.chunk_end;
  const int ne = nblk * kBS + 2 * nS;
  if (!ADJ && st.frozen) return;
  {
    // chunk flags and costs (wave 0)
    const bool need_cost = !ADJ && it == 0;
    int f = 0;
    double F = 0.0;
    if (tid < 64) wave_chunk_sums(K.part_flag_a, K.part_cost_a, c0, c1, need_cost, tid, f, F);
    if (tid == 0) {
      sFail[0] = f;
      if (need_cost) {
        F *= 0.5;
        if (K.vi_cost_a) F += K.vi_cost_a[wi];
        st.cost = F;
        st.init_cost = F;
        if (!isfinite(F)) st.status = 1;
      }
    }
  }
  {
    // eight loads in flight per thread (the system is up to 160 KB); the
    // blocks move from the summed partials' stride kBS to the dense kRS
    const double* src = K.ssum + W.sum_off;
    const int nb = nblk * kBS;
    constexpr int B = 8;
    for (int base = 0; base < ne; base += B * NT) {
      double v[B];
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int e = base + tid + b * NT;
        v[b] = e < ne ? src[e] : 0.0;
      }
#pragma unroll
      for (int b = 0; b < B; ++b) {
        const int e = base + tid + b * NT;
        if (e >= ne) continue;
        if (e < nb) {
          const int blk = e / kBS, r = e - kBS * blk;
          if (r < 36) sS[kRS * blk + r] = v[b];
        } else {
          sS[nblk * kRS + (e - nb)] = v[b];
        }
      }
    }
  }
  __syncthreads();
  if (!ADJ && S.grad_tol > 0) {
    // freeze test at this attempt's linearisation and damping: the reduced
    // right-hand side (summed) and the chunks' landmark gradient maxima; not
    // when a landmark block failed
    double m = 0.0;
    for (int e = tid; e < nS; e += NT) m = fmax(m, fabs(sB[e]));
    for (int c = c0 + tid; c < c1; c += NT) m = fmax(m, K.part_gmax[c]);
    const double gm = block_max<NT>(m, sMax);
    if (tid == 0) {
      sFail[1] = sFail[0] == 0 && gm <= S.grad_tol;
      if (sFail[1]) st.frozen = 1;
    }
    __syncthreads();
    if (sFail[1]) return;
  }
  const double lam = st.lambda;
  const double* poses = (ADJ || st.cur == 0 ? U.poses : K.poses_b) + 12 * W.pose_off;
  if (ADJ) {
    // right-hand side: tangent cotangent of the free poses plus the partials
    for (int i = tid; i < W.n_poses; i += NT) {
      const int f = P.free_slot[W.pose_off + i];
      if (f < 0) continue;
      const double* G = U.grad_poses + 12 * (W.pose_off + i);
      const double* Tp = poses + 12 * i;
      double M[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          M[3 * a + b] = G[4 * a] * Tp[4 * b] + G[4 * a + 1] * Tp[4 * b + 1] +
                         G[4 * a + 2] * Tp[4 * b + 2] + G[4 * a + 3] * Tp[4 * b + 3];
      sB[6 * f + 0] += G[3];
      sB[6 * f + 1] += G[7];
      sB[6 * f + 2] += G[11];
      sB[6 * f + 3] += M[7] - M[5];
      sB[6 * f + 4] += M[2] - M[6];
      sB[6 * f + 5] += M[3] - M[1];
    }
  } else {
    for (int e = tid; e < nS; e += NT) {
      const int f = e / 6, r = e % 6;
      const double d = sD[e];
      sS[kRS * blk_index(f, f, nf) + 7 * r] += lam * (d > 1e-9 ? d : 1e-9);
    }
  }
  __syncthreads();
  // mirror the diagonal blocks (only their upper triangles were accumulated)
  for (int e = tid; e < nf * 36; e += NT) {
    const int f = e / 36, r = (e % 36) / 6, c = e % 6;
    if (c < r) {
      double* D = sS + kRS * blk_index(f, f, nf);
      D[6 * r + c] = D[6 * c + r];
    }
  }
  __syncthreads();

  // Blocked Cholesky S = R^T R on 6x6 blocks (upper block storage), right-
  // looking.  The right-hand side rides along as one more column, so the
  // forward substitution R^T y = b happens inside the factorisation.  Wave 0
  // factors the next diagonal block while the other waves run the trailing
  // update (one step of look-ahead); the back substitution runs in wave 0.
  const int wave = tid >> 6, lane = tid & 63;
  const int lr = lane / 6, lc = lane - 6 * (lane / 6);   // entry of a 6x6 block (lanes 0..35)
  bool failed = sFail[0] != 0;
  if (!failed && nf > 0 && wave == 0) {
    double a = lane < 36 ? sS[kRS * blk_index(0, 0, nf) + lane] : 0.0;
    factor_diag(a, sS + kRS * blk_index(0, 0, nf), sInv, sFail);
  }
  __syncthreads();
  failed = sFail[0] != 0;
  for (int k = 0; k < nf && !failed; ++k) {
    const double* Dk = sS + kRS * blk_index(k, k, nf);
    const double* ik = sInv + 6 * k;
    const int nt = nf - k - 1;
    // panel: R_kj = R_kk^-T S_kj for j > k, one thread per column; the last
    // item is the right-hand side y_k = R_kk^-T b_k
    for (int e = tid; e <= 6 * nt; e += NT) {
      double* B;
      int stride;
      if (e < 6 * nt) {
        B = sS + kRS * blk_index(k, k + 1 + e / 6, nf) + e % 6;
        stride = 6;
      } else {
        B = sB + 6 * k;
        stride = 1;
      }
      double col[6], dku[15], iv[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) col[i] = B[stride * i];
#pragma unroll
      for (int i = 1, q = 0; i < 6; ++i)
#pragma unroll
        for (int m = 0; m < i; ++m, ++q) dku[q] = Dk[6 * m + i];
#pragma unroll
      for (int i = 0; i < 6; ++i) iv[i] = ik[i];
      lds_fence(col);
      lds_fence(dku);
      lds_fence(iv);
      double y[6];
#pragma unroll
      for (int i = 0, q = 0; i < 6; ++i) {
        double v = col[i];
#pragma unroll
        for (int m = 0; m < i; ++m, ++q) v -= dku[q] * y[m];
        y[i] = v * iv[i];
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) B[stride * i] = y[i];
    }
    __syncthreads();
    if (wave == 0) {
      // look-ahead: update and factor the next diagonal block
      if (nt > 0) {
        const double* R = sS + kRS * blk_index(k, k + 1, nf);
        double* Dn = sS + kRS * blk_index(k + 1, k + 1, nf);
        double a = 0.0;
        if (lane < 36) {
          double ra[6], rb[6], dn[1];
#pragma unroll
          for (int m = 0; m < 6; ++m) {
            ra[m] = R[6 * m + lr];
            rb[m] = R[6 * m + lc];
          }
          dn[0] = Dn[lane];
          lds_fence(ra);
          lds_fence(rb);
          lds_fence(dn);
          double acc = 0.0;
#pragma unroll
          for (int m = 0; m < 6; ++m) acc += ra[m] * rb[m];
          a = dn[0] - acc;
        }
        factor_diag(a, Dn, sInv + 6 * (k + 1), sFail);
      }
    } else {
      // trailing update over the npair upper blocks and the nt right-hand
      // side blocks, two items of three rows per block
      const int npair = nt * (nt + 1) / 2 - 1;
      for (int e = tid - 64; e < 2 * (npair + nt); e += NT - 64) trail_item<3>(sS, sB, k, nf, nt, npair, e);
    }
    __syncthreads();
    failed = sFail[0] != 0;
  }
  if (!failed && wave == 0 && nf > 0) {
    // back substitution R x = y in one wave.  Lane l keeps rows 3 l .. 3 l + 2
    // (all three in block row l / 2), so the rows of block k sit in lanes
    // 2 k and 2 k + 1 at register positions known at compile time, and x
    // replaces y there.  A block issues its reads and broadcasts together and
    // waits for them once; the column reads are waited for only after the
    // block's serial chain.
    double y[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) y[t] = 3 * lane + t < nS ? sB[3 * lane + t] : 0.0;
    for (int k = nf - 1; k >= 0; --k) {
      const double* Dk = sS + kRS * blk_index(k, k, nf);
      double dku[15], iv[6], yv[6], bv[18];
#pragma unroll
      for (int i = 0, q = 0; i < 6; ++i)
#pragma unroll
        for (int m = i + 1; m < 6; ++m, ++q) dku[q] = Dk[6 * i + m];
#pragma unroll
      for (int i = 0; i < 6; ++i) iv[i] = sInv[6 * k + i];
      {
        // lanes at or past block row k are not updated; they read block row 0
        const int l = lane < 2 * k ? lane : 0;
        const double* B = sS + kRS * blk_index(l >> 1, k, nf) + 18 * (l & 1);
#pragma unroll
        for (int m = 0; m < 18; m += 2) {
          const double2 b2 = *reinterpret_cast<const double2*>(B + m);
          bv[m] = b2.x;
          bv[m + 1] = b2.y;
        }
      }
#pragma unroll
      for (int i = 0; i < 6; ++i) yv[i] = wave_bcast(y[i % 3], 2 * k + i / 3);
      lds_fence(dku);
      lds_fence(iv);
      lds_fence(yv);
      double x[6];
#pragma unroll
      for (int i = 5; i >= 0; --i) {
        double v = yv[i];
        // dku holds row i's entries m = i + 1 .. 5 at q0(i) .. q0(i) + 4 - i
        const int q0 = 5 * i - i * (i - 1) / 2;
#pragma unroll
        for (int m = i + 1; m < 6; ++m) v -= dku[q0 + m - i - 1] * x[m];
        x[i] = v * iv[i];
      }
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const double d = bv[6 * t] * x[0] + bv[6 * t + 1] * x[1] + bv[6 * t + 2] * x[2] +
                         bv[6 * t + 3] * x[3] + bv[6 * t + 4] * x[4] + bv[6 * t + 5] * x[5];
        y[t] = lane < 2 * k ? y[t] - d : (lane == 2 * k ? x[t] : (lane == 2 * k + 1 ? x[3 + t] : y[t]));
      }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t)
      if (3 * lane + t < nS) sB[3 * lane + t] = y[t];
  }
  __syncthreads();
  double* dp = K.dp + kDpStride * wi;
  for (int e = tid; e < nS; e += NT) dp[e] = failed ? 0.0 : sB[e];
  if (ADJ) {
    if (tid == 0 && U.reports) U.reports[wi].chol_failures = failed ? 1 : 0;
    return;
  }
  if (tid == 0) st.fail = failed ? 1 : 0;
  if (failed) return;
  // candidate poses into the other buffer
  double* cand = (st.cur == 0 ? K.poses_b : U.poses) + 12 * W.pose_off;
  for (int i = tid; i < W.n_poses; i += NT) {
    const int f = P.free_slot[W.pose_off + i];
    const double* Tp = poses + 12 * i;
    double* Tc = cand + 12 * i;
    if (f < 0) {
      for (int k = 0; k < 12; ++k) Tc[k] = Tp[k];
      continue;
    }
    double D[12];
    exp_se3(sB + 6 * f, D);
    for (int a = 0; a < 3; ++a) {
      for (int b = 0; b < 3; ++b)
        Tc[4 * a + b] = D[4 * a] * Tp[b] + D[4 * a + 1] * Tp[4 + b] + D[4 * a + 2] * Tp[8 + b];
      Tc[4 * a + 3] = D[4 * a] * Tp[3] + D[4 * a + 1] * Tp[7] + D[4 * a + 2] * Tp[11] + D[4 * a + 3];
    }
  }
}

// ---------------------------------------------------------------------------
// pass B: back-substitution + candidate cost (LM) / adjoint gather (ADJ)
// ---------------------------------------------------------------------------

template <typename Real, int TP, bool ADJ>
__global__ __launch_bounds__(TP) void k_pass_b(DevPlan P, DevTiles T, DevWork<Real> K, DevUser U,
                                               DevSettings S, int it, int cbase) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int chunk = T.chunk_order[cbase + xcd_chunk(blockIdx.x, gridDim.x)];
  const int wi = T.chunk_window[chunk];
  const WinDev W = P.win[wi];
  const WinState& st = K.state[wi];
  const int tid = threadIdx.x;
  if (!ADJ && (st.fail || st.frozen)) {
    if (tid == 0) {
      K.part_cost_b[chunk] = 0.0;
      K.part_flag_b[chunk] = 0;
      K.part_smax[chunk] = 0.0;
    }
    return;
  }
  const int cur = ADJ ? 0 : st.cur;
  const double lam = ADJ ? 0.0 : st.lambda;
  const double* poses = (cur ? K.poses_b : U.poses) + 12 * W.pose_off;
  const double* points = (cur ? K.points_b : U.points) + 3 * W.point_off;
  const double* cposes = (cur ? U.poses : K.poses_b) + 12 * W.pose_off;
  double* cpoints = (cur ? U.points : K.points_b) + 3 * W.point_off;
  const int nS = 6 * W.n_free;

  double* sPose = reinterpret_cast<double*>(smem);
  double* sCam = sPose + ChunkLds::kPose;
  double* sPoseC = sCam + ChunkLds::kCam;          // 64 * 12 (candidate poses)
  double* sDp = sPoseC + ChunkLds::kPose;          // kDpStride
  double* sLP = sDp + kDpStride;                   // TP * 3 (candidate point / a_l)
  double* sRed = sLP + 3 * TP;                     // 16
  int* sFree = reinterpret_cast<int*>(sRed + 16);  // 64
  int* sFlag = sFree + 64;                         // 4
  Real* sPV = reinterpret_cast<Real*>(sFlag + 4);  // TP * 12: V, g, W^T dp per pair

  load_window(P, W, poses, sPose, sCam, sFree);
  if (!ADJ)
    for (int k = tid; k < W.n_poses * 12; k += TP) sPoseC[k] = cposes[k];
  for (int k = tid; k < nS; k += TP) sDp[k] = K.dp[kDpStride * wi + k];
  if (tid == 0) sFlag[0] = 0;
  __syncthreads();

  double cost = 0.0, smax = 0.0;
  const int t0 = T.chunk_tile_begin[chunk], t1 = T.chunk_tile_begin[chunk + 1];
  const int4* trec = reinterpret_cast<const int4*>(T.tile_rec);
  const int4* prec = reinterpret_cast<const int4*>(T.pair_rec);
  int4 ta = make_int4(0, 0, 0, 0);
  int4 rec = make_int4(0, 0, 0, -1);
  if (t0 < t1) {
    ta = trec[2 * t0];
    if (tid < ta.y) rec = prec[ta.x + tid];
  }
  // A tile's global data is fetched during the tile before it: each pair's
  // point and first observation (after the pair records arrive, behind phase
  // 3), each landmark's pair range and point (behind the whole tile).
  double px = 0, py = 0, pz = 0;
  Real du0 = 0, dv0 = 0, wo0 = 1;
  int cam0 = 0;
  auto fetch_pair = [&](const int4& r, double& x, double& y, double& z, Real& du, Real& dv, Real& wo,
                        int& cam) {
    const double* pt = points + 3 * (r.y - W.point_off);
    x = pt[0];
    y = pt[1];
    z = pt[2];
    cam = P.obs_cam[r.x];
    du = K.du[r.x];
    dv = K.dv[r.x];
    wo = K.w ? K.w[r.x] : (Real)1;
  };
  int lb0 = 0, lb1 = 0;
  double lx = 0, ly = 0, lz = 0;
  auto fetch_lm = [&](int lmt, int& b0, int& b1, double& x, double& y, double& z) {
    b0 = P.lm_pair_begin[lmt];
    b1 = P.lm_pair_begin[lmt + 1];
    const double* pt = points + 3 * (lmt - W.point_off);
    x = pt[0];
    y = pt[1];
    z = pt[2];
  };
  if (t0 < t1) {
    if (tid < ta.y) fetch_pair(rec, px, py, pz, du0, dv0, wo0, cam0);
    if (tid < ta.w) fetch_lm(ta.z + tid, lb0, lb1, lx, ly, lz);
  }
  for (int t = t0; t < t1; ++t) {
    // the tile's pairs in the plan's thread order; q is the pair's index in
    // landmark order (the layout of the per-pair LDS rows)
    const int p0 = ta.x, nP = ta.y, l0 = ta.z, nL = ta.w;
    const int q = (rec.z >> 8) & 255, pose = rec.z & 255, nobs = rec.z >> 16;
    const int slot = rec.w, o0 = rec.x, lm = rec.y;
    const int j = lm - l0;
    int4 nta = ta;
    if (t + 1 < t1) nta = trec[2 * (t + 1)];
    // the next tile's landmarks (their tile record is needed first)
    int nlb0 = 0, nlb1 = 0;
    double nlx = 0, nly = 0, nlz = 0;
    if (t + 1 < t1 && tid < nta.w) fetch_lm(nta.z + tid, nlb0, nlb1, nlx, nly, nlz);

    // ---- phase 1: per pair: W, V, g at the current state and W^T dp
    if (tid < nP) {
      const double* Rt = sPose + 12 * pose;
      double xb[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) xb[a] = Rt[4 * a] * px + Rt[4 * a + 1] * py + Rt[4 * a + 2] * pz + Rt[4 * a + 3];
      Real Rp[9];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Rp[3 * a + b] = (Real)Rt[4 * a + b];
      PairAcc<Real> A;
      pair_zero(A);
      {
        const double* C = sCam + 16 * cam0;
        const Lin<Real> L = linearise<Real>(xb, C, (double)du0, (double)dv0, (double)wo0, S.huber_delta);
        pair_add<Real, ADJ>(A, L, Rp, slot >= 0, C);
      }
      for (int o = o0 + 1; o < o0 + nobs; ++o) {
        const double* C = sCam + 16 * P.obs_cam[o];
        const double wo = K.w ? (double)K.w[o] : 1.0;
        const Lin<Real> L = linearise<Real>(xb, C, (double)K.du[o], (double)K.dv[o], wo,
                                            S.huber_delta);
        pair_add<Real, ADJ>(A, L, Rp, slot >= 0, C);
      }
      Real wtd[3] = {0, 0, 0};
      if (slot >= 0) {
        const double* d = sDp + 6 * slot;
        for (int c = 0; c < 3; ++c) {
          double v = 0.0;
          for (int r = 0; r < 6; ++r) v += (double)A.W[3 * r + c] * d[r];
          wtd[c] = (Real)v;
        }
      }
      for (int k = 0; k < 6; ++k) sPV[12 * q + k] = A.V[k];
      for (int k = 0; k < 3; ++k) sPV[12 * q + 6 + k] = A.gl[k];
      for (int k = 0; k < 3; ++k) sPV[12 * q + 9 + k] = wtd[k];
    }
    __syncthreads();

    // ---- phase 2: per landmark: dl = V*^-1 (c_l - sum W^T dp)
    if (tid < nL) {
      const int lmt = l0 + tid;
      const int q0 = lb0 - p0, q1 = lb1 - p0;
      Real V[6] = {0, 0, 0, 0, 0, 0}, g[3] = {0, 0, 0}, s3[3] = {0, 0, 0};
#pragma unroll 4
      for (int qq = q0; qq < q1; ++qq) {
        for (int k = 0; k < 6; ++k) V[k] += sPV[12 * qq + k];
        for (int k = 0; k < 3; ++k) g[k] += sPV[12 * qq + 6 + k];
        for (int k = 0; k < 3; ++k) s3[k] += sPV[12 * qq + 9 + k];
      }
      Real c[3];
      if (!ADJ) {
        damp3(V, lam);
        for (int k = 0; k < 3; ++k) c[k] = -g[k] - s3[k];
      } else {
        for (int k = 0; k < 3; ++k)
          c[k] = (U.grad_points ? (Real)U.grad_points[3 * lmt + k] : (Real)0) - s3[k];
      }
      LDL3<Real> F;
      ldl3(V, !ADJ, F);
      Real x[3];
      ldl3_solve(F, c, x);
      const double pt[3] = {lx, ly, lz};
      if (!ADJ) {
        double* cp = cpoints + 3 * (lmt - W.point_off);
        for (int k = 0; k < 3; ++k) {
          const double v = pt[k] + (double)x[k];
          sLP[3 * tid + k] = v;
          cp[k] = v;
          smax = fmax(smax, fabs((double)x[k]));
        }
      } else {
        for (int k = 0; k < 3; ++k) sLP[3 * tid + k] = (double)x[k];
      }
    }
    // next tile's pair records (its tile record has arrived by now)
    int4 nrec = make_int4(0, 0, 0, -1);
    if (t + 1 < t1 && tid < nta.y) nrec = prec[nta.x + tid];
    __syncthreads();
    // the next tile's pairs: points and first observations, behind phase 3
    double npx = 0, npy = 0, npz = 0;
    Real ndu = 0, ndv = 0, nwo = 1;
    int ncam = 0;
    if (t + 1 < t1 && tid < nta.y) fetch_pair(nrec, npx, npy, npz, ndu, ndv, nwo, ncam);

    // ---- phase 3: per pair: candidate cost (LM) / per-observation gradients (ADJ)
    if (tid < nP) {
      if (!ADJ) {
        const double* Rt = sPoseC + 12 * pose;
        const double* pt = sLP + 3 * j;
        double xb[3];
        for (int a = 0; a < 3; ++a)
          xb[a] = Rt[4 * a] * pt[0] + Rt[4 * a + 1] * pt[1] + Rt[4 * a + 2] * pt[2] + Rt[4 * a + 3];
        for (int o = o0; o < o0 + nobs; ++o) {
          const bool first = o == o0;   // the first observation is in registers
          const double* C = sCam + 16 * (first ? cam0 : P.obs_cam[o]);
          const double X = C[4] * xb[0] + C[5] * xb[1] + C[6] * xb[2] + C[13];
          const double Y = C[7] * xb[0] + C[8] * xb[1] + C[9] * xb[2] + C[14];
          const double Z = C[10] * xb[0] + C[11] * xb[1] + C[12] * xb[2] + C[15];
          if (!(Z > S.min_depth)) sFlag[0] = 1;
          const double iz = recip_nr(Z);
          const double r0 = C[0] * X * iz - (double)(first ? du0 : K.du[o]);
          const double r1 = C[1] * Y * iz - (double)(first ? dv0 : K.dv[o]);
          double rho, d1, d2;
          huber(r0 * r0 + r1 * r1, S.huber_delta, rho, d1, d2);
          cost += (first ? (double)wo0 : (K.w ? (double)K.w[o] : 1.0)) * rho;
        }
      } else {
        const double* Rt = sPose + 12 * pose;
        double xb[3];
        for (int a = 0; a < 3; ++a) xb[a] = Rt[4 * a] * px + Rt[4 * a + 1] * py + Rt[4 * a + 2] * pz + Rt[4 * a + 3];
        const double* al = sLP + 3 * j;
        const double zero6[6] = {0, 0, 0, 0, 0, 0};
        const double* ap = slot >= 0 ? sDp + 6 * slot : zero6;
        // R_i^T applied on the landmark part: J_l a_l = a . (R_i a_l)
        double Ral[3];
        for (int a = 0; a < 3; ++a)
          Ral[a] = Rt[4 * a] * al[0] + Rt[4 * a + 1] * al[1] + Rt[4 * a + 2] * al[2];
        // pose part: J_p a_p = a . rho + (x_b x a) . phi = a . (rho + phi x x_b)
        double pc[3];
        pc[0] = ap[4] * xb[2] - ap[5] * xb[1];
        pc[1] = ap[5] * xb[0] - ap[3] * xb[2];
        pc[2] = ap[3] * xb[1] - ap[4] * xb[0];
        double v3[3];
        for (int a = 0; a < 3; ++a) v3[a] = ap[a] + pc[a] + Ral[a];
        for (int o = o0; o < o0 + nobs; ++o) {
          const double* C = sCam + 16 * P.obs_cam[o];
          const double wo = K.w ? (double)K.w[o] : 1.0;
          const Lin<Real> L = linearise<Real>(xb, C, (double)K.du[o], (double)K.dv[o], wo,
                                              S.huber_delta);
          const double ja0 = (double)L.a0[0] * v3[0] + (double)L.a0[1] * v3[1] + (double)L.a0[2] * v3[2];
          const double ja1 = (double)L.a1[0] * v3[0] + (double)L.a1[1] * v3[1] + (double)L.a1[2] * v3[2];
          const double r0 = (double)L.r[0], r1 = (double)L.r[1];
          const double rja = r0 * ja0 + r1 * ja1;
          const int u = W.obs_off + P.obs_perm[o];
          U.grad_uv[2 * u] = wo * (L.d1 * ja0 + 2.0 * L.d2 * r0 * rja);
          U.grad_uv[2 * u + 1] = wo * (L.d1 * ja1 + 2.0 * L.d2 * r1 * rja);
          if (U.grad_w) U.grad_w[u] = -L.d1 * rja;
        }
      }
    }
    __syncthreads();
    ta = nta;
    rec = nrec;
    px = npx;
    py = npy;
    pz = npz;
    du0 = ndu;
    dv0 = ndv;
    wo0 = nwo;
    cam0 = ncam;
    lb0 = nlb0;
    lb1 = nlb1;
    lx = nlx;
    ly = nly;
    lz = nlz;
  }
  if (!ADJ) {
    const double tot = block_sum<TP>(cost, sRed);
    if (tid == 0) {
      K.part_cost_b[chunk] = tot;
      K.part_flag_b[chunk] = sFlag[0];
    }
    if (S.step_tol > 0) {
      const double sm = block_max<TP>(smax, sRed);
      if (tid == 0) K.part_smax[chunk] = sm;
    }
  }
}

// ---------------------------------------------------------------------------
// accept / finalize
// ---------------------------------------------------------------------------

template <typename Real>
__global__ void k_accept(DevPlan P, DevTiles T, DevWork<Real> K, DevUser U, DevSettings S, int it, int wbase,
                         int nwin) {
  // one wave per window: the lanes sum the candidate's chunk costs and depth
  // flags, lane 0 decides
  const int i = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= nwin) return;
  const int wi = T.win_order[wbase + i];
  const WinDev W = P.win[wi];
  int depth = 0;
  double F = 0.0;
  wave_chunk_sums(K.part_flag_b, K.part_cost_b, W.chunk_begin, W.chunk_end, true, lane, depth, F);
  // the step's max-norm for the step test: pose tangents and the chunks' point moves
  double sm = 0.0;
  if (S.step_tol > 0) {
    for (int e = lane; e < 6 * W.n_free; e += 64) sm = fmax(sm, fabs(K.dp[kDpStride * wi + e]));
    for (int c = W.chunk_begin + lane; c < W.chunk_end; c += 64) sm = fmax(sm, K.part_smax[c]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sm = fmax(sm, __shfl_xor(sm, off, 64));
  }
  if (lane != 0) return;
  WinState st = K.state[wi];
  ba_iter_trace tr;
  tr.cost = st.cost;
  tr.lambda = st.lambda;
  tr.cand_cost = __builtin_nan("");
  tr.accepted = 0;
  tr.status = 0;
  if (st.frozen) {   // frozen by an earlier attempt or by this one's gradient test
    tr.status = 3;
    if (U.traces) U.traces[(size_t)wi * S.max_iters + it] = tr;
    return;
  }
  bool accept = false;
  if (st.fail) {
    tr.status = 1;
    st.chol_failures++;
  } else {
    if (depth) {
      tr.status = 2;
      st.depth_rejects++;
    } else {
      F *= 0.5;
      if (K.vi_cost_b) F += K.vi_cost_b[wi];
      tr.cand_cost = F;
      st.cand_cost = F;
      accept = F < st.cost;
    }
  }
  if (accept) {
    st.cost = tr.cand_cost;
    st.cur ^= 1;
    st.accepted++;
    st.lambda = fmax(st.lambda / S.lambda_down, S.lambda_min);
    if (S.step_tol > 0 && sm <= S.step_tol) st.frozen = 1;
  } else {
    st.lambda = fmin(st.lambda * S.lambda_up, S.lambda_max);
  }
  tr.accepted = accept ? 1 : 0;
  st.iters++;
  st.fail = 0;
  K.state[wi] = st;
  if (U.traces) U.traces[(size_t)wi * S.max_iters + it] = tr;
}

// Copy the final state into the user's arrays where it sits in the workspace
// buffer, and write the report.  One workgroup per window.
template <typename Real>
__global__ void k_finalize(DevPlan P, DevWork<Real> K, DevUser U, int need_cost) {
  const int wi = blockIdx.x;
  const WinDev W = P.win[wi];
  const WinState st = K.state[wi];
  if (st.cur == 1) {
    for (int k = threadIdx.x; k < 12 * W.n_poses; k += blockDim.x)
      U.poses[12 * W.pose_off + k] = K.poses_b[12 * W.pose_off + k];
    if (K.vi_states)
      for (int k = threadIdx.x; k < 9 * W.n_poses; k += blockDim.x)
        K.vi_states[9 * W.pose_off + k] = K.vi_states_b[9 * W.pose_off + k];
    for (int k = threadIdx.x; k < 3 * W.n_points; k += blockDim.x)
      U.points[3 * W.point_off + k] = K.points_b[3 * W.point_off + k];
  }
  // no attempt ran: the cost comes from the pass-A partials, summed as the
  // first attempt's reduce sums them
  int fdummy = 0;
  double F = 0.0;
  if (need_cost && threadIdx.x < 64)
    wave_chunk_sums(K.part_flag_a, K.part_cost_a, W.chunk_begin, W.chunk_end, true, threadIdx.x, fdummy, F);
  if (threadIdx.x == 0) {
    ba_report r;
    double c0 = st.init_cost, cf = st.cost;
    if (need_cost) c0 = cf = 0.5 * F;
    r.initial_cost = c0;
    r.final_cost = cf;
    r.final_lambda = st.lambda;
    r.iters = st.iters;
    r.accepted = st.accepted;
    r.chol_failures = st.chol_failures;
    r.depth_rejects = st.depth_rejects;
    r.status = (need_cost && !isfinite(c0)) ? 1 : st.status;
    r.reserved = 0;
    U.reports[wi] = r;
  }
}

// ---------------------------------------------------------------------------
// host-side launch helpers (instantiated here, called by the ABI layer)
// ---------------------------------------------------------------------------

template <typename Real, int TP>
size_t pass_a_lds(int np, int nc, int nf, int list_bytes, bool adj) {
  return PassALds<Real, TP>::bytes(np, nc, nf, list_bytes, adj);
}

template <typename Real, int TP>
size_t pass_b_lds() {
  return (2 * ChunkLds::kPose + ChunkLds::kCam + kDpStride + 3 * TP + 16) * sizeof(double) +
         (64 + 4) * sizeof(int) + (size_t)TP * 12 * sizeof(Real);
}

// The reduce kernel's LDS: the reduced system of the largest window.
size_t reduce_lds(int max_nf) {
  const int nblk = max_nf * (max_nf + 1) / 2;
  return (size_t)(nblk * kRS + 18 * max_nf + 11) * sizeof(double);
}

constexpr int kReduceThreads = 512;

template <typename Real, int TP, bool ADJ>
hipError_t set_attrs() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pass_a<Real, TP, ADJ>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_pass_b<Real, TP, ADJ>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_reduce<Real, kReduceThreads, ADJ>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

// Pass A over the size classes, each launch with the LDS its largest window
// needs.  With side streams, the largest class and the next one each run on a
// side stream, concurrently with the rest on the launch stream: the classes
// share the CUs, so one class's long workgroups fill the others' launch tails,
// and workgroups of a small class fit beside one of the largest class in the
// LDS of a CU (measured on the 256-window batch: +21 % LM attempts per second
// over the four launches in sequence; merging classes of equal occupancy into
// one launch gained 6 %).
struct PassAGroup {
  int begin, n;
  size_t lds;
  int stream;   // 0: the launch stream, k > 0: side stream k - 1
};

template <typename Real, int TP, bool ADJ>
int pass_a_groups(const LaunchArgs& A, PassAGroup* g) {
  int ng = 0;
  for (int c = 0; c < kClasses; ++c) {
    const int n = A.cls_begin[c + 1] - A.cls_begin[c];
    if (n <= 0) continue;
    const size_t lds = pass_a_lds<Real, TP>(A.dims.np, A.dims.nc, A.cls_nf[c], A.list_bytes, ADJ);
    g[ng++] = PassAGroup{A.cls_begin[c], n, lds, 0};
  }
  if (A.side_stream && ng >= 2) {
    g[ng - 1].stream = 1;
    if (ng >= 3) g[ng - 2].stream = 2;
  }
  return ng;
}

template <typename Real, int TP, bool ADJ>
hipError_t launch_pass_a(const LaunchArgs& A, const DevWork<Real>& K, int it) {
  static_assert(kSideStreams >= 2, "pass A uses two side streams");
  PassAGroup g[kClasses];
  const int ng = pass_a_groups<Real, TP, ADJ>(A, g);
  const hipStream_t main = (hipStream_t)A.stream;
  const hipStream_t* side = (const hipStream_t*)A.side_stream;
  const hipEvent_t* join = (const hipEvent_t*)A.ev_join;
  bool used[kSideStreams + 1] = {};
  for (int k = 0; k < ng; ++k) used[g[k].stream] = true;
  bool fork = false;
  for (int s = 1; s <= kSideStreams; ++s) fork = fork || used[s];
  hipError_t e = hipSuccess;
  if (fork && (e = hipEventRecord((hipEvent_t)A.ev_fork, main)) != hipSuccess) return e;
  for (int s = 1; s <= kSideStreams; ++s)
    if (used[s] && (e = hipStreamWaitEvent(side[s - 1], (hipEvent_t)A.ev_fork, 0)) != hipSuccess) return e;
  for (int k = ng - 1; k >= 0; --k)   // side launches first
    if (g[k].stream)
      hipLaunchKernelGGL((k_pass_a<Real, TP, ADJ>), dim3(g[k].n), dim3(TP), g[k].lds, side[g[k].stream - 1], A.plan,
                         A.tiles, K, A.user, A.settings, it, g[k].begin, A.dims);
  for (int k = 0; k < ng; ++k)
    if (!g[k].stream)
      hipLaunchKernelGGL((k_pass_a<Real, TP, ADJ>), dim3(g[k].n), dim3(TP), g[k].lds, main, A.plan, A.tiles, K,
                         A.user, A.settings, it, g[k].begin, A.dims);
  for (int s = 1; s <= kSideStreams; ++s)
    if (used[s]) {
      if ((e = hipEventRecord(join[s - 1], side[s - 1])) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(main, join[s - 1], 0)) != hipSuccess) return e;
    }
  return hipGetLastError();
}


// The stages after pass A of one LM attempt for the windows [wb, wb + nwin) of
// win_order (at most nf free poses each) and their chunks [cb, cb + nch) of
// chunk_order, on stream st.
template <typename Real, int TP, bool ADJ>
void launch_stages(const LaunchArgs& A, const DevWork<Real>& K, int it, int wb, int nwin, int cb, int nch, int nf,
                   int slices, hipStream_t st) {
  if (nwin <= 0) return;
  const size_t lb = pass_b_lds<Real, TP>(), lr = reduce_lds(nf);
  hipLaunchKernelGGL(k_sum<Real>, dim3(nwin, slices), dim3(256), 0, st, A.plan, A.tiles, K, wb);
  if (!ADJ && A.vi) launch_vi_lin(*static_cast<const ViArgs*>(A.vi), wb, nwin, st);
  hipLaunchKernelGGL((k_reduce<Real, kReduceThreads, ADJ>), dim3(nwin), dim3(kReduceThreads), lr, st, A.plan, A.tiles,
                     K, A.user, A.settings, it, wb);
  if (!ADJ && A.vi) launch_vi_cand(*static_cast<const ViArgs*>(A.vi), wb, nwin, st);
  if (nch > 0)
    hipLaunchKernelGGL((k_pass_b<Real, TP, ADJ>), dim3(nch), dim3(TP), lb, st, A.plan, A.tiles, K, A.user, A.settings,
                       it, cb);
  if (!ADJ)
    hipLaunchKernelGGL(k_accept<Real>, dim3((nwin + 3) / 4), dim3(256), 0, st, A.plan, A.tiles, K, A.user,
                       A.settings, it, wb, nwin);
}

// One pass-A launch of size class c on stream st.
template <typename Real, int TP, bool ADJ>
void launch_pass_a_class(const LaunchArgs& A, const DevWork<Real>& K, int it, int c, hipStream_t st) {
  const int n = A.cls_begin[c + 1] - A.cls_begin[c];
  if (n <= 0) return;
  const size_t lds = pass_a_lds<Real, TP>(A.dims.np, A.dims.nc, A.cls_nf[c], A.list_bytes, ADJ);
  hipLaunchKernelGGL((k_pass_a<Real, TP, ADJ>), dim3(n), dim3(TP), lds, st, A.plan, A.tiles, K, A.user, A.settings, it,
                     A.cls_begin[c], A.dims);
}

// The windows of one size class never meet those of another, so with side
// streams every class runs its whole LM loop (pass A, sum, reduce, pass B,
// acceptance per attempt) as a chain of its own, forked once after the set-up
// and joined once before the final copy: the largest class on side stream 1,
// the next on side stream 2, the smaller ones one after the other on the
// launch stream (as pass A's split in launch_pass_a).  The small grids of the
// reduce and pass B then overlap with other classes' pass A instead of every
// class waiting for the slowest one in each attempt (256-window batch: 271 k
// -> 285 k LM attempts/s; four chains on four streams: 279 k; the smallest
// class on a side stream with a larger one: 242-273 k).
struct ClassChains {
  int n = 0, nside = 0;
  int cls[kClasses];            // the classes that hold windows, ascending
  hipStream_t st[kClasses];     // the stream of each
};

// The chains of a launch, or n = 0 when everything runs on the launch stream
// (no side streams, or fewer than two classes).
inline ClassChains class_chains(const LaunchArgs& A) {
  ClassChains C;
  int ncls = 0;
  for (int c = 0; c < kClasses; ++c)
    if (A.cls_win_begin[c + 1] > A.cls_win_begin[c]) C.cls[ncls++] = c;
  if (!A.side_stream || ncls < 2) return C;
  const hipStream_t* side = (const hipStream_t*)A.side_stream;
  C.n = ncls;
  C.nside = ncls >= 3 ? 2 : 1;   // classes on side streams: the largest nside
  for (int k = 0; k < ncls; ++k) {
    const int r = ncls - 1 - k;  // rank from the largest class
    C.st[k] = r < C.nside ? side[r] : (hipStream_t)A.stream;
  }
  return C;
}

inline hipError_t fork_chains(const LaunchArgs& A, const ClassChains& C) {
  const hipStream_t* side = (const hipStream_t*)A.side_stream;
  hipError_t e = hipEventRecord((hipEvent_t)A.ev_fork, (hipStream_t)A.stream);
  for (int r = 0; r < C.nside && e == hipSuccess; ++r) e = hipStreamWaitEvent(side[r], (hipEvent_t)A.ev_fork, 0);
  return e;
}

inline hipError_t join_chains(const LaunchArgs& A, const ClassChains& C) {
  const hipStream_t* side = (const hipStream_t*)A.side_stream;
  const hipEvent_t* join = (const hipEvent_t*)A.ev_join;
  hipError_t e = hipSuccess;
  for (int r = 0; r < C.nside && e == hipSuccess; ++r) {
    e = hipEventRecord(join[r], side[r]);
    if (e == hipSuccess) e = hipStreamWaitEvent((hipStream_t)A.stream, join[r], 0);
  }
  return e;
}

// One attempt of class C.cls[k] on its chain's stream.
template <typename Real, int TP, bool ADJ>
void launch_class_attempt(const LaunchArgs& A, const DevWork<Real>& K, int it, const ClassChains& C, int k) {
  const int c = C.cls[k];
  launch_pass_a_class<Real, TP, ADJ>(A, K, it, c, C.st[k]);
  launch_stages<Real, TP, ADJ>(A, K, it, A.cls_win_begin[c], A.cls_win_begin[c + 1] - A.cls_win_begin[c],
                               A.cls_begin[c], A.cls_begin[c + 1] - A.cls_begin[c], A.cls_win_nf[c],
                               A.cls_sum_slices[c], C.st[k]);
}

template <typename Real, int TP>
hipError_t run_solve(const LaunchArgs& A, const DevWork<Real>& K) {
  const int nw = A.plan.n_windows, nc = A.tiles.n_chunks;
  const hipStream_t main = (hipStream_t)A.stream;
  hipLaunchKernelGGL(k_init<Real>, dim3((nw + 63) / 64), dim3(64), 0, main, A.plan, K, A.settings);
  hipLaunchKernelGGL(k_pack<Real>, dim3(nc), dim3(256), 0, main, A.plan, A.tiles, K, A.user);
  const int iters = A.settings.max_iters;
  const ClassChains C = class_chains(A);
  hipError_t e = hipSuccess;
  if (C.n > 0 && iters > 0) {
    if ((e = fork_chains(A, C)) != hipSuccess) return e;
    for (int it = 0; it < iters; ++it)
      for (int k = C.n - 1; k >= 0; --k) launch_class_attempt<Real, TP, false>(A, K, it, C, k);
    if ((e = join_chains(A, C)) != hipSuccess) return e;
  } else {
    for (int it = 0; it < iters; ++it) {
      if ((e = launch_pass_a<Real, TP, false>(A, K, it)) != hipSuccess) return e;
      launch_stages<Real, TP, false>(A, K, it, 0, nw, 0, nc, A.max_nf, A.sum_slices, main);
    }
  }
  if (iters == 0 && (e = launch_pass_a<Real, TP, false>(A, K, 0)) != hipSuccess)   // the report still needs the input cost
    return e;
  hipLaunchKernelGGL(k_finalize<Real>, dim3(nw), dim3(256), 0, main, A.plan, K, A.user, iters == 0 ? 1 : 0);
  return hipGetLastError();
}

// The adjoint's single pass, in the same class chains as a solve.
template <typename Real, int TP>
hipError_t run_adjoint(const LaunchArgs& A, const DevWork<Real>& K) {
  const int nw = A.plan.n_windows, nc = A.tiles.n_chunks;
  const hipStream_t main = (hipStream_t)A.stream;
  hipLaunchKernelGGL(k_init<Real>, dim3((nw + 63) / 64), dim3(64), 0, main, A.plan, K, A.settings);
  hipLaunchKernelGGL(k_pack<Real>, dim3(nc), dim3(256), 0, main, A.plan, A.tiles, K, A.user);
  const ClassChains C = class_chains(A);
  hipError_t e = hipSuccess;
  if (C.n > 0) {
    if ((e = fork_chains(A, C)) != hipSuccess) return e;
    for (int k = C.n - 1; k >= 0; --k) launch_class_attempt<Real, TP, true>(A, K, 0, C, k);
    if ((e = join_chains(A, C)) != hipSuccess) return e;
  } else {
    if ((e = launch_pass_a<Real, TP, true>(A, K, 0)) != hipSuccess) return e;
    launch_stages<Real, TP, true>(A, K, 0, 0, nw, 0, nc, A.max_nf, A.sum_slices, main);
  }
  return hipGetLastError();
}

// The attempt-by-attempt sequence (pass A's classes forked and joined within
// each attempt, the other stages over all windows on the launch stream) with
// HIP events between the stages: the summed device time of each stage
// (pass_a, reduce, pass_b, accept) in ms, for the roofline figures of the
// benchmark.  Synchronises on the stream.
template <typename Real, int TP>
hipError_t run_solve_timed(const LaunchArgs& A, const DevWork<Real>& K, double* stage_ms) {
  const int nw = A.plan.n_windows, nc = A.tiles.n_chunks;
  const hipStream_t main = (hipStream_t)A.stream;
  const size_t lb = pass_b_lds<Real, TP>(), lr = reduce_lds(A.max_nf);
  const int iters = A.settings.max_iters;
  const int nev = 4 * iters + 1;
  hipEvent_t* ev = new hipEvent_t[nev];
  for (int k = 0; k < nev; ++k) (void)hipEventCreate(&ev[k]);
  hipLaunchKernelGGL(k_init<Real>, dim3((nw + 63) / 64), dim3(64), 0, main, A.plan, K, A.settings);
  hipLaunchKernelGGL(k_pack<Real>, dim3(nc), dim3(256), 0, main, A.plan, A.tiles, K, A.user);
  (void)hipEventRecord(ev[0], main);
  hipError_t e = hipSuccess;
  for (int it = 0; it < iters && e == hipSuccess; ++it) {
    e = launch_pass_a<Real, TP, false>(A, K, it);
    (void)hipEventRecord(ev[4 * it + 1], main);
    hipLaunchKernelGGL(k_sum<Real>, dim3(nw, A.sum_slices), dim3(256), 0, main, A.plan, A.tiles, K, 0);
    hipLaunchKernelGGL((k_reduce<Real, kReduceThreads, false>), dim3(nw), dim3(kReduceThreads), lr, main, A.plan,
                       A.tiles, K, A.user, A.settings, it, 0);
    (void)hipEventRecord(ev[4 * it + 2], main);
    hipLaunchKernelGGL((k_pass_b<Real, TP, false>), dim3(nc), dim3(TP), lb, main, A.plan, A.tiles, K, A.user,
                       A.settings, it, 0);
    (void)hipEventRecord(ev[4 * it + 3], main);
    hipLaunchKernelGGL(k_accept<Real>, dim3((nw + 3) / 4), dim3(256), 0, main, A.plan, A.tiles, K, A.user,
                       A.settings, it, 0, nw);
    (void)hipEventRecord(ev[4 * it + 4], main);
  }
  hipLaunchKernelGGL(k_finalize<Real>, dim3(nw), dim3(256), 0, main, A.plan, K, A.user, 0);
  if (e == hipSuccess) e = hipGetLastError();
  if (e == hipSuccess) e = hipEventSynchronize(ev[nev - 1]);
  for (int k = 0; k < 4; ++k) stage_ms[k] = 0.0;
  for (int it = 0; it < iters && e == hipSuccess; ++it)
    for (int k = 0; k < 4; ++k) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ev[4 * it + k], ev[4 * it + k + 1]);
      stage_ms[k] += ms;
    }
  for (int k = 0; k < nev; ++k) (void)hipEventDestroy(ev[k]);
  delete[] ev;
  return e;
}

// explicit instantiations used by the ABI layer
template size_t pass_a_lds<double, 64>(int, int, int, int, bool);
template size_t pass_a_lds<double, 256>(int, int, int, int, bool);
template size_t pass_a_lds<float, 64>(int, int, int, int, bool);
template size_t pass_a_lds<float, 256>(int, int, int, int, bool);
template size_t pass_b_lds<double, 64>();
template size_t pass_b_lds<double, 256>();
template size_t pass_b_lds<float, 64>();
template size_t pass_b_lds<float, 256>();
template hipError_t set_attrs<double, 64, false>();
template hipError_t set_attrs<double, 256, false>();
template hipError_t set_attrs<float, 64, false>();
template hipError_t set_attrs<float, 256, false>();
template hipError_t set_attrs<double, 64, true>();
template hipError_t set_attrs<double, 256, true>();
template hipError_t set_attrs<float, 64, true>();
template hipError_t set_attrs<float, 256, true>();
template hipError_t run_solve<double, 64>(const LaunchArgs&, const DevWork<double>&);
template hipError_t run_solve<double, 256>(const LaunchArgs&, const DevWork<double>&);
template hipError_t run_solve<float, 64>(const LaunchArgs&, const DevWork<float>&);
template hipError_t run_solve<float, 256>(const LaunchArgs&, const DevWork<float>&);
template hipError_t run_solve_timed<double, 64>(const LaunchArgs&, const DevWork<double>&, double*);
template hipError_t run_solve_timed<double, 256>(const LaunchArgs&, const DevWork<double>&, double*);
template hipError_t run_solve_timed<float, 64>(const LaunchArgs&, const DevWork<float>&, double*);
template hipError_t run_solve_timed<float, 256>(const LaunchArgs&, const DevWork<float>&, double*);
template hipError_t run_adjoint<double, 64>(const LaunchArgs&, const DevWork<double>&);
template hipError_t run_adjoint<double, 256>(const LaunchArgs&, const DevWork<double>&);
template hipError_t run_adjoint<float, 64>(const LaunchArgs&, const DevWork<float>&);
template hipError_t run_adjoint<float, 256>(const LaunchArgs&, const DevWork<float>&);

}  // namespace ba
