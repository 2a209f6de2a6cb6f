// Structures shared by the host launcher and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/ba.h"
#include "plan.hpp"

namespace ba {

// Upper block (i <= j) of an nf x nf block matrix, row-major over the triangle.
__host__ __device__ __forceinline__ int blk_index(int i, int j, int nf) {
  return i * nf - (i * (i - 1)) / 2 + (j - i);
}

// The pair (i, j), i <= j, of upper block e of an n x n block matrix.
__device__ __forceinline__ void upper_pair(int e, int n, int& i, int& j) {
  const float b = 2.0f * n + 1.0f;
  int r = (int)((b - sqrtf(b * b - 8.0f * e)) * 0.5f);
  r = r < 0 ? 0 : (r > n - 1 ? n - 1 : r);
  while (r > 0 && r * n - r * (r - 1) / 2 > e) --r;
  while (r + 1 < n && (r + 1) * n - (r + 1) * r / 2 <= e) ++r;
  i = r;
  j = e - (r * n - r * (r - 1) / 2) + r;
}

// Per-window structure, uploaded once per plan.
struct WinDev {
  int32_t n_poses, n_points, n_cams, n_free;
  int32_t pose_off, point_off, cam_off, obs_off;   // first pose / landmark / camera / observation
  int32_t pair_off, chunk_begin, chunk_end, sum_off;   // sum_off: summed system in the workspace
  int32_t sum_groups;   // chunk groups of k_sum (see sum_groups())
};

// Per-window LM state, in the workspace.
struct WinState {
  double lambda;      // damping of the next attempt
  double cost;        // F at the current state
  double cand_cost;   // F at the last candidate
  double init_cost;   // F at the input state
  int32_t cur;        // which buffer holds the current state: 0 user arrays, 1 workspace
  int32_t fail;       // this attempt met a non-positive pivot
  int32_t accepted, chol_failures, depth_rejects, iters, status;
  int32_t frozen;     // a freeze test has stopped the window (no more attempts)
};

// Read-only plan arrays (batch-global indices unless stated).
struct DevPlan {
  const WinDev* win;
  const int32_t* free_slot;       // per pose: free slot in its window or -1
  const double* cam;              // per camera: fx fy cx cy R(9) t(3)
  const int32_t* lm_pair_begin;   // per landmark + 1: first pair
  const uint8_t* lm_nfree;        // per landmark: free pairs (stored first)
  const int32_t* pair_obs_begin;  // per pair + 1: first observation (plan order)
  const int32_t* pair_lm;         // per pair: landmark
  const uint8_t* pair_pose;       // per pair: window-local pose
  const uint8_t* obs_cam;         // per observation: window-local camera
  const int32_t* obs_perm;        // per observation: window-local user index
  int32_t n_windows;
};

struct DevTiles {
  const int32_t* chunk_order;     // chunks grouped by size class
  const int32_t* win_order;       // windows grouped by size class
  const int32_t* pair_rec;        // 4 per pair position (thread order of its tile)
  const int32_t* tile_rec;        // 8 per tile
  const uint32_t* lists;          // per tile: segment words then products
  const int32_t* tile_lm_begin;
  const int32_t* chunk_window;
  const int32_t* chunk_tile_begin;
  const int64_t* chunk_part_off;
  int32_t n_chunks;
};

template <typename Real>
struct DevWork {
  Real* du;                 // per observation, plan order: u - cx
  Real* dv;                 // v - cy
  Real* w;                  // weight, NULL when every weight is 1
  double* poses_b;          // second state buffer (candidate / current)
  double* points_b;
  WinState* state;
  double* dp;               // per window, kDpStride doubles: the reduced-system solution
  double* ssum;             // per window: the chunk partials summed in FP64
  Real* part;               // chunk partials of S, the reduced rhs and diag(U)
  double* part_cost_a;      // per chunk: sum w rho at the current state
  double* part_cost_b;      // per chunk: sum w rho at the candidate
  int32_t* part_flag_a;     // per chunk: a landmark block was not positive definite
  int32_t* part_flag_b;     // per chunk: a candidate depth <= min_depth
  double* part_gmax;        // per chunk: largest |landmark gradient| (LM solves)
  double* part_smax;        // per chunk: largest |landmark step| (step_tol > 0)
  // visual-inertial solves only (NULL otherwise): per window the IMU cost at
  // the current state and at the candidate; the velocities and biases (user
  // buffer and workspace buffer, 9 per pose)
  double* vi_cost_a;
  double* vi_cost_b;
  double* vi_states;
  double* vi_states_b;
};

struct DevUser {
  double* poses;
  double* points;
  const double* obs_uv;
  const double* obs_w;
  ba_report* reports;
  ba_iter_trace* traces;
  const double* grad_poses;
  const double* grad_points;
  double* grad_uv;
  double* grad_w;
};

struct DevSettings {
  double lambda_init, lambda_up, lambda_down, lambda_min, lambda_max;
  double huber_delta, min_depth;
  double grad_tol, step_tol;   // freeze tests (0: off)
  int32_t max_iters;
  int32_t pad;
};

constexpr int kDpStride = 192;

// k_sum: a 256-thread workgroup sums kSumE entries per thread of a window's
// chunk partials, split into G groups of 256 / G threads; group g adds the
// window's chunks g, g + G, g + 2G, ... in that order and the G group sums are
// added in group order.  G depends only on the window's chunk count (so a
// window sums in the same order alone or in any batch): about 16 chunks per
// group, a power of two up to 16.
constexpr int kSumE = 4;
inline int sum_groups(int n_chunks) {
  int g = 1;
  while (g < 16 && g * 16 < n_chunks) g *= 2;
  return g;
}
inline int sum_slice_entries(int groups) { return 256 / groups * kSumE; }

constexpr int kSideStreams = 2;   // side streams of the size classes

// Dimensions of the window caches in LDS (largest in the launch).
struct LdsDims {
  int np, nc;
};

// Everything one launch sequence needs (built by the ABI layer).
struct LaunchArgs {
  DevPlan plan;
  DevTiles tiles;
  DevUser user;
  DevSettings settings;
  int max_nf;
  int cls_begin[kClasses + 1];   // chunk_order ranges of the size classes
  int cls_win_begin[kClasses + 1];   // win_order ranges of the size classes
  int cls_win_nf[kClasses];      // largest free-pose count of each class's windows
  int cls_nf[kClasses];          // largest free-pose count of each class
  LdsDims dims;                  // largest pose / camera count of the batch
  int list_bytes;                // largest per-tile product list (segments + products)
  int max_cpw;                   // largest number of chunks of one window
  int cls_sum_slices[kClasses];  // k_sum workgroups per window of each class
  int sum_slices;                // the same over all windows
  void* stream;                  // hipStream_t
  // The side streams of the size classes (hipStream_t[kSideStreams], or NULL
  // to run everything on `stream`), the event that forks them from `stream`
  // and the events (hipEvent_t[kSideStreams]) that join them back.
  void* side_stream;
  void* ev_fork;
  void* ev_join;
  // visual-inertial solves: the IMU stages' arguments (const ViArgs*), or NULL
  const void* vi;
};

}  // namespace ba
