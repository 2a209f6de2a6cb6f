// Interface between the C ABI layer and the triangulation kernel (tri.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"

namespace ba {

struct TriArgs {
  const double* cams;              // n_cams * 16: fx fy cx cy, R_cb, t_cb (device)
  int n_cams;
  int n_points;
  int n_poses;
  long long n_obs;
  const int32_t* point_obs_begin;  // n_points + 1 (device)
  const double* poses;             // n_poses * 12, base-from-world, read only
  const int32_t* obs_pose;         // n_obs
  const int32_t* obs_cam;          // n_obs or NULL
  const double* obs_uv;            // n_obs * 2
  const double* obs_w;             // n_obs or NULL
  double* points;                  // n_points * 3, out
  ba_report* reports;              // n_points or NULL
  ba_iter_trace* traces;           // n_points * max_iters or NULL
  DevSettings settings;
  void* stream;
};

template <typename Real>
hipError_t run_triangulate(const TriArgs& A);

}  // namespace ba
