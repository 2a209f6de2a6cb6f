// Interface between the C ABI layer and the motion-only kernels (pnp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"

namespace ba {

struct PnpArgs {
  const double* cams;              // n_cams * 16: fx fy cx cy, R_cb, t_cb (device)
  int n_cams;
  int n_frames;
  long long n_obs, n_points;
  const int32_t* frame_obs_begin;  // n_frames + 1 (device)
  double* poses;                   // n_frames * 12, in/out
  const double* points;            // n_points * 3
  const int32_t* obs_point;        // n_obs
  const int32_t* obs_cam;          // n_obs or NULL
  const double* obs_uv;            // n_obs * 2
  const double* obs_w;             // n_obs or NULL
  const double* frame_transform;   // n_frames * 12 (T^mw) or NULL
  ba_report* reports;              // n_frames or NULL
  ba_iter_trace* traces;           // n_frames * max_iters or NULL
  DevSettings settings;
  int waves_per_frame;             // 1, 2 or 4
  void* stream;
};

// Waves per frame for a launch of n_frames frames and n_obs observations.
int pnp_waves_per_frame(int n_frames, long long n_obs);

template <typename Real>
hipError_t run_pnp(const PnpArgs& A);

}  // namespace ba
