// Pose-graph optimisation (paper Sec. 2.3, Eq. 15): the interface of the
// kernels (pgo.hip) to the ABI layer; the host plan is in pgo_plan.hpp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "device.hpp"
#include "pgo_plan.hpp"

namespace ba {

// Device copy of the plan's tables.
struct PgoDev {
  int n_poses, n_edges, n_free, n_levels, n_blocks;
  const int32_t *col_of_pose, *pose_of_col, *lev_ptr, *blk_ptr, *blk_row;
  const int32_t *upd_ptr, *upd_a, *upd_b, *fwd_ptr, *fwd_blk, *fwd_col;
  const int32_t *asm_ptr, *asm_edge, *rhs_ptr, *rhs_edge, *edge_i, *edge_j;
  const int32_t *blk_col, *chunk_ptr, *chunk_blk, *fchunk_ptr, *fchunk_col;
  const int32_t *chunk_ab, *fchunk_bc;
  int n_chunks, n_fchunks;
  int n_wide;
};

struct PgoArgs {
  PgoDev G;
  PgoWork W;
  double* poses;          // n_poses * 12 world-from-base, in/out
  const double* deltas;   // n_edges * 12
  const double* edge_w;   // n_edges or NULL
  ba_report* report;      // 1 or NULL
  ba_iter_trace* traces;  // max_iters or NULL
  DevSettings settings;
  void* stream;
  const int* wide_tasks;  // HOST, 3 * G.n_wide launch sizes
};

hipError_t run_pgo(const PgoArgs& A);

}  // namespace ba
