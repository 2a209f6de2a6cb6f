// Visual-inertial extension of the window solve (vi.hip): record layouts and
// launchers used by the window solver's launch sequence.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"

namespace ba {

// Preintegrated factor record (doubles), one per consecutive pair of states:
// dR (9), dv (3), dp (3), dT, the bias Jacobians J_Rg, J_vg, J_va, J_pg, J_pa
// (9 each, row-major), the bias estimates it was integrated at (b^a, b^w),
// and the 15x15 information of (r_R, r_v, r_p, r_ba, r_bg).
constexpr int kPreDR = 0, kPreDv = 9, kPreDp = 12, kPreDT = 15, kPreJRg = 16, kPreJvg = 25, kPreJva = 34,
              kPreJpg = 43, kPreJpa = 52, kPreBa = 61, kPreBg = 64, kPreInfo = 67;
constexpr int kPreStride = BA_VI_PREINT_DOUBLES;
static_assert(kPreInfo + 225 <= kPreStride, "preintegration record stride");
constexpr int kViMaxStates = 24;            // keyframes of a visual-inertial window
constexpr int kViFactorStride = 960;        // workspace doubles per factor (linearisation record)

// Everything the VI kernels need for one launch (single-window solves).
struct ViArgs {
  const WinDev* win;
  const int32_t* win_order;
  const int32_t* free_slot;
  WinState* state;
  double* poses;          // user poses (one state buffer)
  double* poses_b;        // workspace poses (the other)
  double* states;         // user velocities and biases, 9 per pose (v, b^a, b^w)
  double* states_b;       // workspace copy (the other buffer)
  const double* preint;   // n_poses - 1 records, factor f joins poses f and f + 1
  double* rec;            // workspace: factor records, then A^-1 [H_yx | g_y]
  double* ssum;           // the summed reduced system (S, rhs, diag)
  const double* dp;       // the poses' step
  int32_t* part_flag_a;   // chunk flags of pass A (a failed elimination sets one)
  double* cost_a;         // per window: IMU cost at the current state
  double* cost_b;         // per window: IMU cost at the candidate
  double g[3];            // gravity, world frame
  int max_factors;        // IMU factors of the largest window (grid of the factor kernel)
};

hipError_t launch_vi_preint(int n_factors, const int32_t* sample_begin, const double* gyro, const double* accel,
                            double dt, const double* bias_bar, const double* noise, double* out, hipStream_t st);
void launch_vi_lin(const ViArgs& V, int wbase, int nwin, hipStream_t st);
void launch_vi_cand(const ViArgs& V, int wbase, int nwin, hipStream_t st);

// Workspace doubles of the VI records of a window of n poses and nf free poses.
inline size_t vi_rec_doubles(int n_poses, int n_free) {
  return (size_t)kViFactorStride * (n_poses - 1) + (size_t)9 * n_poses * (6 * n_free + 1);
}

}  // namespace ba
