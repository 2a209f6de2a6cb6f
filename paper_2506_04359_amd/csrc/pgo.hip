// gfx950 pose-graph optimisation (paper Sec. 2.3, Eq. 15): LM over the
// world-from-base poses T_i minimising 1/2 sum_e w_e |Log(D_ij^-1 T_i^-1 T_j)|^2.
//
// Per LM attempt (besides one k_pgo_wide launch per wide level of the
// elimination tree):
//   k_pgo_edges  one thread per edge at the candidate poses: r = Log(E),
//                E = D^-1 T_i^-1 T_j, B = J_l(r)^-1 Ad(D^-1 T_i^-1) (so dr/dxi_j
//                = B, dr/dxi_i = -B for the left perturbation), and w B^T B,
//                w B^T r, w |r|^2 into an edge buffer (two buffers: the current
//                linearisation and the candidate's)
//   k_pgo_decide     one workgroup: the candidate's cost (fixed-order sum),
//                    accept iff it strictly drops, lambda, trace
//   k_pgo_assemble   the damped normal equations gathered from the current
//                    edge buffer into the factor's blocks, -g into y
//   k_pgo_wide       the wide levels of the sparse block Cholesky (see below)
//   k_pgo_factor     one 1024-thread workgroup: the narrow levels (left-
//                    looking: each column gathers its updates, factors its
//                    diagonal block in registers, solves its panel; the
//                    forward substitution rides along), then back substitution
//   k_pgo_candidate  the next candidate Exp(d_i) T_i
// Every sum has a fixed order and nothing uses atomics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.hpp"
#include "geometry.hpp"
#include "pgo.hpp"

namespace ba {

constexpr int kPgoEdgeThreads = 256;
constexpr int kPgoStepThreads = 1024;

// 3x3 helpers (row-major)
__device__ __forceinline__ void mm3(const double* A, const double* B, double* C) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) C[3 * a + b] = A[3 * a] * B[b] + A[3 * a + 1] * B[3 + b] + A[3 * a + 2] * B[6 + b];
}
__device__ __forceinline__ void skew3(const double* v, double* K) {
  K[0] = 0.0; K[1] = -v[2]; K[2] = v[1];
  K[3] = v[2]; K[4] = 0.0; K[5] = -v[0];
  K[6] = -v[1]; K[7] = v[0]; K[8] = 0.0;
}
// C = A B for 3x4 transforms; inverse of a 3x4 transform
__device__ __forceinline__ void tcompose(const double* A, const double* B, double* C) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int b = 0; b < 3; ++b) C[4 * a + b] = A[4 * a] * B[b] + A[4 * a + 1] * B[4 + b] + A[4 * a + 2] * B[8 + b];
    C[4 * a + 3] = A[4 * a] * B[3] + A[4 * a + 1] * B[7] + A[4 * a + 2] * B[11] + A[4 * a + 3];
  }
}
__device__ __forceinline__ void tinverse(const double* T, double* I) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int b = 0; b < 3; ++b) I[4 * a + b] = T[4 * b + a];
    I[4 * a + 3] = -(T[a] * T[3] + T[4 + a] * T[7] + T[8 + a] * T[11]);
  }
}

// Log of a rotation: phi with Exp(phi) = R.  theta = atan2(|v|, (tr R - 1) / 2)
// with v the vee of the antisymmetric part (sin(theta) times the axis); the
// axis from the symmetric part near theta = pi.
__device__ __forceinline__ void log_so3(const double* T /*3x4*/, double* phi) {
  const double v[3] = {0.5 * (T[9] - T[6]), 0.5 * (T[2] - T[8]), 0.5 * (T[4] - T[1])};
  double c = 0.5 * (T[0] + T[5] + T[10] - 1.0);
  c = fmin(1.0, fmax(-1.0, c));
  const double s = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  const double th = atan2(s, c);
  if (c > -0.999) {
    // theta / sin(theta); series below theta = 1e-3
    const double t2 = th * th;
    const double f = th < 1e-3 ? 1.0 + t2 * (1.0 / 6.0 + t2 * (7.0 / 360.0)) : th / s;
    phi[0] = f * v[0];
    phi[1] = f * v[1];
    phi[2] = f * v[2];
    return;
  }
  // (R + R^T) / 2 = c I + (1 - c) a a^T
  const double Md[3] = {T[0] - c, T[5] - c, T[10] - c};
  int k = 0;
  if (Md[1] > Md[k]) k = 1;
  if (Md[2] > Md[k]) k = 2;
  const double ic = 1.0 / (1.0 - c);
  double a[3];
  a[k] = sqrt(fmax(Md[k] * ic, 0.0));
  const double ia = 1.0 / a[k];
#pragma unroll
  for (int m = 0; m < 3; ++m)
    if (m != k) a[m] = 0.5 * (T[4 * m + k] + T[4 * k + m]) * ic * ia;
  const double sg = (a[0] * v[0] + a[1] * v[1] + a[2] * v[2]) < 0.0 ? -1.0 : 1.0;
  phi[0] = sg * th * a[0];
  phi[1] = sg * th * a[1];
  phi[2] = sg * th * a[2];
}

// Inverse of the SO(3) left Jacobian: I - K/2 + d K^2, d = 1/th^2 -
// cot(th/2) / (2 th) (series below th = 0.1).
__device__ __forceinline__ void jl_inv_so3(const double* phi, double* Ji) {
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
  mm3(K, K, K2);
#pragma unroll
  for (int k = 0; k < 9; ++k) Ji[k] = ((k % 4 == 0) ? 1.0 : 0.0) - 0.5 * K[k] + d * K2[k];
}

// Top-right block Q of the SE(3) left Jacobian J_l(rho, phi) =
// sum_n ad^n / (n+1)!: with ad^n = [[K^n, X_n], [0, K^n]], X_{n+1} = K X_n +
// P K^n (P = rho^), Q = sum_{n >= 1} X_n / (n+1)!; summed until the bound
// th^n n |rho| / (n+1)! is below 1e-18 (at most 40 terms).
__device__ __forceinline__ void jl_q_se3(const double* rho, const double* phi, double* Q) {
  double K[9], P[9], Kn[9], X[9], t1[9], t2[9];
  skew3(phi, K);
  skew3(rho, P);
  const double th = sqrt(phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]);
  const double nr = sqrt(rho[0] * rho[0] + rho[1] * rho[1] + rho[2] * rho[2]);
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    Kn[k] = (k % 4 == 0) ? 1.0 : 0.0;   // K^0
    X[k] = 0.0;                          // X_0
    Q[k] = 0.0;
  }
  double fact = 1.0;    // (n+1)!
  double thn = 1.0;     // th^n
  for (int n = 0; n < 40; ++n) {
    // X_{n+1} = K X_n + P K^n, K^{n+1} = K K^n
    mm3(K, X, t1);
    mm3(P, Kn, t2);
#pragma unroll
    for (int k = 0; k < 9; ++k) X[k] = t1[k] + t2[k];
    mm3(K, Kn, t1);
#pragma unroll
    for (int k = 0; k < 9; ++k) Kn[k] = t1[k];
    fact *= (double)(n + 2);   // (n+2)!
#pragma unroll
    for (int k = 0; k < 9; ++k) Q[k] += X[k] / fact;
    thn *= th;
    if (thn * (n + 1) * nr / fact < 1e-18 && n >= 1) break;
  }
}

__global__ __launch_bounds__(kPgoEdgeThreads) void k_pgo_edges(PgoArgs A, int init) {
  const int e = blockIdx.x * kPgoEdgeThreads + threadIdx.x;
  if (e >= A.G.n_edges) return;
  const int cur = A.W.istate[0];
  double* out = A.W.edge[init ? 0 : 1 - cur] + 28 * (long long)e;
  const double* P = init ? A.poses : A.W.cand;
  const double* Ti = P + 12 * (long long)A.G.edge_i[e];
  const double* Tj = P + 12 * (long long)A.G.edge_j[e];
  const double* D = A.deltas + 12 * (long long)e;
  const double w = A.edge_w ? A.edge_w[e] : 1.0;
  double Di[12], Tii[12], X[12], E[12];
  tinverse(D, Di);
  tinverse(Ti, Tii);
  tcompose(Di, Tii, X);   // D^-1 T_i^-1
  tcompose(X, Tj, E);     // D^-1 T_i^-1 T_j
  // r = Log(E) = (J^-1 t, phi)
  double phi[3], Ji[9], r[6];
  log_so3(E, phi);
  jl_inv_so3(phi, Ji);
#pragma unroll
  for (int a = 0; a < 3; ++a) r[a] = Ji[3 * a] * E[3] + Ji[3 * a + 1] * E[7] + Ji[3 * a + 2] * E[11];
  r[3] = phi[0];
  r[4] = phi[1];
  r[5] = phi[2];
  // B = J_l(r)^-1 Ad(X) = [[M, N], [0, M]]: M = J^-1 R_X, N = J^-1 (t_X^ R_X - Q M)
  double Q[9], R[9], M[9], tX[9], K1[9], QM[9], N[9], tmp[9];
  jl_q_se3(r, phi, Q);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) R[3 * a + b] = X[4 * a + b];
  mm3(Ji, R, M);
  const double tv[3] = {X[3], X[7], X[11]};
  skew3(tv, tX);
  mm3(tX, R, K1);
  mm3(Q, M, QM);
#pragma unroll
  for (int k = 0; k < 9; ++k) tmp[k] = K1[k] - QM[k];
  mm3(Ji, tmp, N);
  // B (6x6) explicitly, then w B^T B (upper), w B^T r, w |r|^2
  double B[36];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      B[6 * a + b] = M[3 * a + b];
      B[6 * a + 3 + b] = N[3 * a + b];
      B[6 * (a + 3) + b] = 0.0;
      B[6 * (a + 3) + 3 + b] = M[3 * a + b];
    }
  int k = 0;
#pragma unroll
  for (int a = 0; a < 6; ++a)
#pragma unroll
    for (int b = a; b < 6; ++b, ++k) {
      double v = 0.0;
#pragma unroll
      for (int m = 0; m < 6; ++m) v += B[6 * m + a] * B[6 * m + b];
      out[k] = w * v;
    }
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    double v = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) v += B[6 * m + a] * r[m];
    out[21 + a] = w * v;
  }
  double rr = 0.0;
#pragma unroll
  for (int m = 0; m < 6; ++m) rr += r[m] * r[m];
  out[27] = w * rr;
}

// upper-triangle index of (a, b) in a 6x6 symmetric block
__device__ __forceinline__ int up6(int a, int b) {
  const int lo = a < b ? a : b, hi = a < b ? b : a;
  return 6 * lo - lo * (lo - 1) / 2 + hi - lo;
}

// Decision on the candidate just evaluated (mode 1), or the start (mode 0):
// the cost summed in a fixed order, accept iff it strictly drops, lambda,
// trace, the accepted poses, and the report after the last attempt.
__global__ __launch_bounds__(kPgoStepThreads) void k_pgo_decide(PgoArgs A, int mode, int it, int last) {
  __shared__ double sRed[kPgoStepThreads];
  const int tid = threadIdx.x;
  const PgoDev& G = A.G;
  const PgoWork& W = A.W;
  const DevSettings S = A.settings;
  double* st = W.state;      // 0 F, 1 lambda, 2 F0
  int32_t* ist = W.istate;   // 0 current buffer, 1 candidate valid, 2 accepted, 3 chol failures
  const int cur0 = mode == 0 ? 0 : ist[0];
  const int ev = mode == 0 ? 0 : 1 - cur0;
  double s = 0.0;
  for (int e = tid; e < G.n_edges; e += kPgoStepThreads) s += W.edge[ev][28 * (long long)e + 27];
  sRed[tid] = s;
  __syncthreads();
  for (int h = kPgoStepThreads / 2; h > 0; h >>= 1) {
    if (tid < h) sRed[tid] += sRed[tid + h];
    __syncthreads();
  }
  const double Fe = 0.5 * sRed[0];
  double F, lam;
  if (mode == 0) {
    F = Fe;
    lam = S.lambda_init;
    if (tid == 0) {
      st[0] = F;
      st[1] = lam;
      st[2] = F;
      ist[0] = 0;
      ist[2] = 0;
      ist[3] = 0;
    }
  } else {
    F = st[0];
    lam = st[1];
    const bool valid = ist[1] != 0;
    const bool accept = valid && Fe < F;
    if (tid == 0 && A.traces) {
      ba_iter_trace tr;
      tr.cost = F;
      tr.lambda = lam;
      tr.cand_cost = valid ? Fe : __builtin_nan("");
      tr.status = valid ? 0 : 1;
      tr.accepted = accept ? 1 : 0;
      A.traces[it] = tr;
    }
    if (accept) {
      for (int k = tid; k < 12 * G.n_poses; k += kPgoStepThreads) A.poses[k] = W.cand[k];
      F = Fe;
    }
    lam = accept ? fmax(lam / S.lambda_down, S.lambda_min) : fmin(lam * S.lambda_up, S.lambda_max);
    if (tid == 0) {
      st[0] = F;
      st[1] = lam;
      if (accept) {
        ist[0] = 1 - cur0;
        ist[2] += 1;
      }
    }
  }
  if (last && tid == 0 && A.report) {
    ba_report r;
    r.initial_cost = mode == 0 ? F : st[2];
    r.final_cost = F;
    r.final_lambda = lam;
    r.iters = S.max_iters;
    r.accepted = mode == 0 ? 0 : ist[2];
    r.chol_failures = mode == 0 ? 0 : ist[3];
    r.depth_rejects = 0;
    r.status = isfinite(r.initial_cost) ? 0 : 1;
    r.reserved = 0;
    *A.report = r;
  }
}

// The damped normal equations gathered from the current edge buffer into the
// factor's blocks (one thread per block row), and -g into y.
__global__ __launch_bounds__(kPgoEdgeThreads) void k_pgo_assemble(PgoArgs A) {
  const PgoDev& G = A.G;
  const PgoWork& W = A.W;
  const int t = blockIdx.x * kPgoEdgeThreads + threadIdx.x;
  const double* EB = W.edge[W.istate[0]];
  if (t == 0) W.istate[4] = 0;   // pivot failure flag of the factorisation that follows
  const int nb6 = G.n_blocks * 6;
  if (t < nb6) {
    const int b = t / 6, a = t % 6;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int q = G.asm_ptr[b]; q < G.asm_ptr[b + 1]; ++q) {
      const int ce = G.asm_edge[q];
      const double* x = EB + 28 * (long long)(ce >> 1);
      const double sg = (ce & 1) ? -1.0 : 1.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) v[c] += sg * x[up6(a, c)];
    }
    if (G.blk_ptr[G.blk_row[b]] == b) {   // diagonal block: damping
      const double lam = W.state[1];
      v[a] += lam * fmax(v[a], 1e-9);
    }
    double* out = W.L + 36 * (long long)b + 6 * a;
#pragma unroll
    for (int c = 0; c < 6; ++c) out[c] = v[c];
  } else if (t < nb6 + G.n_free) {
    const int c = t - nb6;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int q = G.rhs_ptr[c]; q < G.rhs_ptr[c + 1]; ++q) {
      const int ce = G.rhs_edge[q];
      const double* x = EB + 28 * (long long)(ce >> 1) + 21;
      const double sg = (ce & 1) ? -1.0 : 1.0;
#pragma unroll
      for (int a = 0; a < 6; ++a) v[a] += sg * x[a];
    }
#pragma unroll
    for (int a = 0; a < 6; ++a) W.y[6 * c + a] = v[a];
  }
}

// Sparse block Cholesky by levels of the elimination tree.  Per level:
// (1) every chunk of at most kPgoChunk updates L_rk L_ck^T of a block (and of
// forward updates L_ck y_k of a right-hand side) is summed by its own thread
// into a partial; (2) one wave per column subtracts its partials in chunk
// order, factors the diagonal block in registers, finishes the forward step
// and solves the column's panel rows.  A wide level is one launch with a
// workgroup per column (its chunks, then its first wave does the rest); the
// narrow ones run in one workgroup, where the partials are first subtracted
// entry-parallel.  A failed pivot sets istate[4].  Back substitution from the
// top level down, six threads per column.
// Phase (1) over the update chunks [q0, q1) and forward chunks [f0, f1).
__device__ __forceinline__ void pgo_phase1_range(const PgoDev& G, const PgoWork& W, int q0, int q1, int f0, int f1,
                                                 int t0, int stride) {
  double* fpart = W.part + 36 * (long long)G.n_chunks;
  const int nq = (q1 - q0) * 36;
  for (int t = t0; t < nq + (f1 - f0) * 6; t += stride) {
    if (t < nq) {
      const int q = q0 + t / 36, e = t % 36, a = e / 6, c = e % 6;
      // the chunk's block pairs in one read (-1 past the list's end; those
      // entries read the first pair and add nothing)
      const int32_t* ab = G.chunk_ab + 2 * kPgoChunk * (long long)q;
      int ia[kPgoChunk], ib[kPgoChunk];
#pragma unroll
      for (int k = 0; k < kPgoChunk; ++k) {
        ia[k] = ab[k];
        ib[k] = ab[kPgoChunk + k];
      }
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < kPgoChunk; ++k) {
        const bool on = ia[k] >= 0;
        const double* La = W.L + 36 * (long long)(on ? ia[k] : ia[0]) + 6 * a;
        const double* Lb = W.L + 36 * (long long)(on ? ib[k] : ib[0]) + 6 * c;
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < 6; ++m) s += La[m] * Lb[m];
        acc += on ? s : 0.0;
      }
      W.part[36 * (long long)q + e] = acc;
    } else {
      const int fq = f0 + (t - nq) / 6, a = (t - nq) % 6;
      const int32_t* bc = G.fchunk_bc + 2 * kPgoChunk * (long long)fq;
      int ib[kPgoChunk], ik[kPgoChunk];
#pragma unroll
      for (int k = 0; k < kPgoChunk; ++k) {
        ib[k] = bc[k];
        ik[k] = bc[kPgoChunk + k];
      }
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < kPgoChunk; ++k) {
        const bool on = ib[k] >= 0;
        const double* Lf = W.L + 36 * (long long)(on ? ib[k] : ib[0]) + 6 * a;
        const double* yk = W.y + 6 * (on ? ik[k] : ik[0]);
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < 6; ++m) s += Lf[m] * yk[m];
        acc += on ? s : 0.0;
      }
      fpart[6 * (long long)fq + a] = acc;
    }
  }
}

// Index ranges of level l: columns, blocks, update chunks, forward chunks.
struct PgoLevel {
  int c0, c1, b0, b1, q0, q1, f0, f1;
};
__device__ __forceinline__ PgoLevel pgo_level(const PgoDev& G, int l) {
  PgoLevel v;
  v.c0 = G.lev_ptr[l];
  v.c1 = G.lev_ptr[l + 1];
  v.b0 = G.blk_ptr[v.c0];
  v.b1 = G.blk_ptr[v.c1];
  v.q0 = G.chunk_ptr[v.b0];
  v.q1 = G.chunk_ptr[v.b1];
  v.f0 = G.fchunk_ptr[v.c0];
  v.f1 = G.fchunk_ptr[v.c1];
  return v;
}

// Phase (1) of a level (all its columns' chunks).
__device__ __forceinline__ void pgo_phase1(const PgoDev& G, const PgoWork& W, const PgoLevel& v, int t0, int stride) {
  pgo_phase1_range(G, W, v.q0, v.q1, v.f0, v.f1, t0, stride);
}

// The level's partials subtracted from its blocks and right-hand sides, one
// entry per thread, in chunk order (the narrow levels' variant of the sums
// that phases 2 and 3 otherwise do per column / row).
__device__ __forceinline__ void pgo_phase1b(const PgoDev& G, const PgoWork& W, const PgoLevel& v, int t0,
                                            int stride) {
  const int c0 = v.c0, c1 = v.c1, b0 = v.b0, b1 = v.b1;
  const double* fpart = W.part + 36 * (long long)G.n_chunks;
  const int nb = (b1 - b0) * 36;
  for (int t = t0; t < nb + (c1 - c0) * 6; t += stride) {
    if (t < nb) {
      const int b = b0 + t / 36, e = t % 36;
      const int q0 = G.chunk_ptr[b], q1 = G.chunk_ptr[b + 1];
      if (q0 == q1) continue;
      double v = W.L[36 * (long long)b + e];
      int q = q0;
      for (; q + 4 <= q1; q += 4) {   // four reads in flight, subtracted in order
        double p[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) p[k] = W.part[36 * (long long)(q + k) + e];
#pragma unroll
        for (int k = 0; k < 4; ++k) v -= p[k];
      }
      for (; q < q1; ++q) v -= W.part[36 * (long long)q + e];
      W.L[36 * (long long)b + e] = v;
    } else {
      const int c = c0 + (t - nb) / 6, a = (t - nb) % 6;
      const int q0 = G.fchunk_ptr[c], q1 = G.fchunk_ptr[c + 1];
      if (q0 == q1) continue;
      double v = W.y[6 * c + a];
      int q = q0;
      for (; q + 4 <= q1; q += 4) {
        double p[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) p[k] = fpart[6 * (long long)(q + k) + a];
#pragma unroll
        for (int k = 0; k < 4; ++k) v -= p[k];
      }
      for (; q < q1; ++q) v -= fpart[6 * (long long)q + a];
      W.y[6 * c + a] = v;
    }
  }
}

// Phases 2 and 3 of a level with one wave per column: every lane factors the
// column's diagonal block in registers (the same arithmetic in each lane) and
// finishes the forward step, then the lanes solve the column's panel rows.
// With SUM the chunk partials are subtracted here (the wide levels).
template <bool SUM>
__device__ __forceinline__ void pgo_phase23(const PgoDev& G, const PgoWork& W, int c0, int c1, int w0, int nw,
                                            int lane, int* sfail = nullptr) {
  const double* fpart = W.part + 36 * (long long)G.n_chunks;
  for (int c = c0 + w0; c < c1; c += nw) {
    const int bd = G.blk_ptr[c];
    double* Lc = W.L + 36 * (long long)bd;
    double m[36], yc[6];
#pragma unroll
    for (int k = 0; k < 36; ++k) m[k] = Lc[k];
#pragma unroll
    for (int a = 0; a < 6; ++a) yc[a] = W.y[6 * c + a];
    if constexpr (SUM) {
      // two chunks' partials read before either is subtracted (in order)
      const int q1 = G.chunk_ptr[bd + 1];
      int q = G.chunk_ptr[bd];
      for (; q + 2 <= q1; q += 2) {
        double p0[36], p1[36];
#pragma unroll
        for (int k = 0; k < 36; ++k) {
          p0[k] = W.part[36 * (long long)q + k];
          p1[k] = W.part[36 * (long long)(q + 1) + k];
        }
#pragma unroll
        for (int k = 0; k < 36; ++k) m[k] = (m[k] - p0[k]) - p1[k];
      }
      for (; q < q1; ++q)
#pragma unroll
        for (int k = 0; k < 36; ++k) m[k] -= W.part[36 * (long long)q + k];
      for (int q = G.fchunk_ptr[c]; q < G.fchunk_ptr[c + 1]; ++q)
#pragma unroll
        for (int a = 0; a < 6; ++a) yc[a] -= fpart[6 * (long long)q + a];
    }
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double d = m[7 * k];
#pragma unroll
      for (int q = 0; q < k; ++q) d -= m[6 * k + q] * m[6 * k + q];
      ok = ok && d > 0.0 && isfinite(d);
      const double lk = sqrt(fmax(d, 1e-300)), il = 1.0 / lk;
      m[7 * k] = lk;
#pragma unroll
      for (int i = k + 1; i < 6; ++i) {
        double v = m[6 * i + k];
#pragma unroll
        for (int q = 0; q < k; ++q) v -= m[6 * i + q] * m[6 * k + q];
        m[6 * i + k] = v * il;
      }
    }
    if (!ok) {
      if (lane == 0) {
        W.istate[4] = 1;
        if (sfail) *sfail = 1;
      }
      continue;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double v = yc[k];
#pragma unroll
      for (int q = 0; q < k; ++q) v -= m[6 * k + q] * yc[q];
      yc[k] = v / m[7 * k];
    }
    // panel rows (every lane has read the diagonal block above)
    const int nrow = (G.blk_ptr[c + 1] - bd - 1) * 6;
    for (int t = lane; t < nrow; t += 64) {
      const int b = bd + 1 + t / 6, a = t % 6;
      double* row = W.L + 36 * (long long)b + 6 * a;
      double x[6];
#pragma unroll
      for (int k = 0; k < 6; ++k) x[k] = row[k];
      if constexpr (SUM) {
        const int q1 = G.chunk_ptr[b + 1];
        int q = G.chunk_ptr[b];
        for (; q + 4 <= q1; q += 4) {   // four chunks' rows in flight, in order
          double p[4][6];
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int k = 0; k < 6; ++k) p[j][k] = W.part[36 * (long long)(q + j) + 6 * a + k];
#pragma unroll
          for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int k = 0; k < 6; ++k) x[k] -= p[j][k];
        }
        for (; q < q1; ++q)
#pragma unroll
          for (int k = 0; k < 6; ++k) x[k] -= W.part[36 * (long long)q + 6 * a + k];
      }
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        double v = x[k];
#pragma unroll
        for (int q = 0; q < k; ++q) v -= x[q] * m[6 * k + q];
        x[k] = v / m[7 * k];
      }
#pragma unroll
      for (int k = 0; k < 6; ++k) row[k] = x[k];
    }
    if (lane == 0) {
#pragma unroll
      for (int k = 0; k < 36; ++k) Lc[k] = m[k];
#pragma unroll
      for (int a = 0; a < 6; ++a) W.y[6 * c + a] = yc[a];
    }
  }
}

// One wide level, one workgroup per column: its update and forward chunks
// (phase 1), then its first wave subtracts them, factors and solves the
// panel (phases 2 and 3).  Columns of a level are independent, so a level is
// one launch.
__global__ __launch_bounds__(kPgoEdgeThreads) void k_pgo_wide(PgoArgs A, int l) {
  const PgoDev& G = A.G;
  const int c = G.lev_ptr[l] + blockIdx.x;
  const int bA = G.blk_ptr[c], bB = G.blk_ptr[c + 1];
  pgo_phase1_range(G, A.W, G.chunk_ptr[bA], G.chunk_ptr[bB], G.fchunk_ptr[c], G.fchunk_ptr[c + 1], threadIdx.x,
                   kPgoEdgeThreads);
  __syncthreads();
  if (threadIdx.x < 64)
    pgo_phase23<true>(G, A.W, G.lev_ptr[l], G.lev_ptr[l + 1], blockIdx.x, gridDim.x, threadIdx.x);
}

// Levels [l0, n_levels) in one workgroup, then the back substitution.
__global__ __launch_bounds__(kPgoStepThreads) void k_pgo_factor(PgoArgs A, int l0) {
  const int tid = threadIdx.x;
  const PgoDev& G = A.G;
  const PgoWork& W = A.W;
  // a failed pivot of the wide levels (earlier launches) or of this one,
  // mirrored in LDS so that the level loop reads no flag from memory
  __shared__ int sFail;
  // the narrow levels' index ranges, read once (level by level in parallel)
  // instead of by every phase of every level
  constexpr int kLevCache = 128;
  __shared__ PgoLevel sLv[kLevCache];
  const int nlv = G.n_levels - l0;
  const bool cached = nlv <= kLevCache;
  if (tid == 0) sFail = W.istate[4];
  if (cached)
    for (int i = tid; i < nlv; i += kPgoStepThreads) sLv[i] = pgo_level(G, l0 + i);
  __syncthreads();
  for (int l = l0; l < G.n_levels; ++l) {
    if (sFail) break;
    const PgoLevel lv = cached ? sLv[l - l0] : pgo_level(G, l);
    pgo_phase1(G, W, lv, tid, kPgoStepThreads);
    __syncthreads();
    pgo_phase1b(G, W, lv, tid, kPgoStepThreads);
    __syncthreads();
    pgo_phase23<false>(G, W, lv.c0, lv.c1, tid >> 6, kPgoStepThreads / 64, tid & 63, &sFail);
    __syncthreads();
  }
  if (sFail) {
    if (tid == 0) {
      W.istate[1] = 0;
      W.istate[3] += 1;
    }
    return;
  }
  // back substitution, x_c = L_cc^-T (y_c - sum over the column's
  // off-diagonal blocks of L_rc^T x_r), the blocks in order: six threads per
  // column, one per row of x_c, each summing its row with two blocks' loads in
  // flight; then every thread of the column's group solves the 6x6 triangle
  // from the six sums (through LDS) and keeps its own row
  __shared__ double sV[kPgoStepThreads];
  constexpr int kCols = kPgoStepThreads / 6;   // columns per pass
  for (int l = G.n_levels - 1; l >= 0; --l) {
    const int c0 = G.lev_ptr[l], c1 = G.lev_ptr[l + 1];
    for (int base = c0; base < c1; base += kCols) {
      const int a = tid % 6, c = base + tid / 6;
      const bool act = tid < 6 * kCols && c < c1;
      double v = 0.0;
      if (act) {
        v = W.y[6 * c + a];
        const int b0 = G.blk_ptr[c] + 1, b1 = G.blk_ptr[c + 1];
        for (int b = b0; b < b1; b += 2) {
          int bk[2], rk[2];
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            bk[k] = min(b + k, b1 - 1);
            rk[k] = G.blk_row[bk[k]];
          }
          double lv[2][6], xv[2][6];
#pragma unroll
          for (int k = 0; k < 2; ++k)
#pragma unroll
            for (int m = 0; m < 6; ++m) {
              lv[k][m] = W.L[36 * (long long)bk[k] + 6 * m + a];
              xv[k][m] = W.x[6 * rk[k] + m];
            }
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            double t = 0.0;
#pragma unroll
            for (int m = 0; m < 6; ++m) t += lv[k][m] * xv[k][m];
            if (b + k < b1) v -= t;
          }
        }
      }
      sV[tid] = v;
      __syncthreads();
      if (act) {
        double vv[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) vv[q] = sV[tid - a + q];
        const double* Lc = W.L + 36 * (long long)G.blk_ptr[c];
#pragma unroll
        for (int k = 5; k >= 0; --k) {
          double s = vv[k];
#pragma unroll
          for (int q = k + 1; q < 6; ++q) s -= Lc[6 * q + k] * vv[q];
          vv[k] = s / Lc[7 * k];
        }
        double mine = vv[0];
#pragma unroll
        for (int q = 1; q < 6; ++q) mine = a == q ? vv[q] : mine;
        W.x[6 * c + a] = mine;
      }
      __syncthreads();
    }
  }
  if (tid == 0) W.istate[1] = 1;
}

// Candidate poses Exp(d_i) T_i for the free poses (the others copied); a
// failed factorisation leaves the current poses.
__global__ __launch_bounds__(kPgoEdgeThreads) void k_pgo_candidate(PgoArgs A) {
  const int i = blockIdx.x * kPgoEdgeThreads + threadIdx.x;
  if (i >= A.G.n_poses) return;
  const int c = A.G.col_of_pose[i];
  const double* T = A.poses + 12 * (long long)i;
  double* out = A.W.cand + 12 * (long long)i;
  if (c < 0 || A.W.istate[1] == 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) out[k] = T[k];
  } else {
    double Dx[12];
    exp_se3(A.W.x + 6 * c, Dx);
    tcompose(Dx, T, out);
  }
}

hipError_t run_pgo(const PgoArgs& A) {
  hipStream_t s = (hipStream_t)A.stream;
  const int eb = (A.G.n_edges + kPgoEdgeThreads - 1) / kPgoEdgeThreads;
  const int ab = (A.G.n_blocks * 6 + A.G.n_free + kPgoEdgeThreads - 1) / kPgoEdgeThreads;
  const int pb = (A.G.n_poses + kPgoEdgeThreads - 1) / kPgoEdgeThreads;
  const int n_it = A.settings.max_iters;
  auto prepare = [&]() {
    // the assembly also clears the pivot-failure flag, so it runs even when
    // there is nothing to gather
    hipLaunchKernelGGL(k_pgo_assemble, dim3(ab > 0 ? ab : 1), dim3(kPgoEdgeThreads), 0, s, A);
    for (int l = 0; l < A.G.n_wide; ++l) {
      const int* w = A.wide_tasks + 3 * l;   // w[1]: the level's columns
      if (w[1] > 0) hipLaunchKernelGGL(k_pgo_wide, dim3(w[1]), dim3(kPgoEdgeThreads), 0, s, A, l);
    }
    hipLaunchKernelGGL(k_pgo_factor, dim3(1), dim3(kPgoStepThreads), 0, s, A, A.G.n_wide);
    hipLaunchKernelGGL(k_pgo_candidate, dim3(pb), dim3(kPgoEdgeThreads), 0, s, A);
  };
  if (eb > 0) hipLaunchKernelGGL(k_pgo_edges, dim3(eb), dim3(kPgoEdgeThreads), 0, s, A, 1);
  hipLaunchKernelGGL(k_pgo_decide, dim3(1), dim3(kPgoStepThreads), 0, s, A, 0, -1, n_it == 0 ? 1 : 0);
  if (n_it > 0) prepare();
  for (int it = 0; it < n_it; ++it) {
    if (eb > 0) hipLaunchKernelGGL(k_pgo_edges, dim3(eb), dim3(kPgoEdgeThreads), 0, s, A, 0);
    hipLaunchKernelGGL(k_pgo_decide, dim3(1), dim3(kPgoStepThreads), 0, s, A, 1, it, it + 1 == n_it ? 1 : 0);
    if (it + 1 < n_it) prepare();
  }
  return hipGetLastError();
}

}  // namespace ba
