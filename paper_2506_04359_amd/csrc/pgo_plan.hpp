// Pose-graph optimisation (paper Sec. 2.3, Eq. 15): host plan of the sparse
// block Cholesky and the workspace carve.  Plain C++ (no HIP), so that it can
// be built and sanitised on the host alone.
#pragma once

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace ba {

// Host plan of one pose graph over its free poses.  Columns of the block
// factor L are numbered in elimination order, grouped by level of the
// elimination tree (every column after its children); a column's blocks are
// its diagonal block followed by its off-diagonal blocks in increasing row.
struct PgoPlan {
  int n_poses = 0, n_edges = 0, n_free = 0, n_levels = 0;
  std::vector<int32_t> col_of_pose;   // n_poses: column of a free pose, -1 when fixed
  std::vector<int32_t> pose_of_col;   // n_free
  std::vector<int32_t> lev_ptr;       // n_levels + 1: columns of each level
  std::vector<int32_t> blk_ptr;       // n_free + 1: blocks of each column
  std::vector<int32_t> blk_row;       // n_blocks: row (column index) of each block
  std::vector<int32_t> upd_ptr;       // n_blocks + 1: updates L_rk L_ck^T into block (r, c)
  std::vector<int32_t> upd_a, upd_b;  //   block ids of L_rk and L_ck
  std::vector<int32_t> fwd_ptr;       // n_free + 1: forward updates y_c -= L_ck y_k
  std::vector<int32_t> fwd_blk, fwd_col;
  std::vector<int32_t> asm_ptr;       // n_blocks + 1: edge terms gathered into each block
  std::vector<int32_t> asm_edge;      //   edge * 2 + (1 when subtracted)
  std::vector<int32_t> rhs_ptr;       // n_free + 1: edge terms gathered into each RHS
  std::vector<int32_t> rhs_edge;      //   edge * 2 + (1 when subtracted)
  std::vector<int32_t> edge_i, edge_j;
  // the update and forward lists cut into chunks of kPgoChunk entries, each
  // summed by its own thread: chunks of block b are [chunk_ptr[b],
  // chunk_ptr[b+1]), chunk_blk the block of a chunk; the same for the forward
  // lists of the columns
  std::vector<int32_t> blk_col;       // n_blocks: column of each block
  // the first n_wide levels run each phase over the whole GPU; wide_tasks
  // holds their task counts (phase 1, 2, 3) per level
  int n_wide = 0;
  std::vector<int32_t> wide_tasks;
  std::vector<int32_t> chunk_ptr, chunk_blk, fchunk_ptr, fchunk_col;
  // per chunk its kPgoChunk block pairs (L_rk ids, then L_ck ids) and per
  // forward chunk its (block, column) pairs, -1 past the list's end: a
  // chunk's thread reads its whole list at once
  std::vector<int32_t> chunk_ab, fchunk_bc;
  int n_blocks() const { return (int)blk_row.size(); }
};

constexpr int kPgoChunk = 4;

// Builds the plan; returns an error message (empty on success).
std::string build_pgo_plan(int32_t n_poses, int32_t n_edges, const int32_t* edge_i,
                           const int32_t* edge_j, const uint8_t* pose_fixed, PgoPlan& P);

// Workspace carved by the solve (FP64 unless noted).
struct PgoWork {
  double* edge[2];    // n_edges * 28: w B^T B (21, upper), w B^T r (6), w |r|^2
  double* cand;       // n_poses * 12 candidate poses
  double* L;          // n_blocks * 36 factor blocks (row-major)
  double* y;          // n_free * 6 right-hand side / forward solution
  double* x;          // n_free * 6 step
  double* part;       // n_chunks * 36 + n_fchunks * 6 partial sums of the update chunks
  double* state;      // 8: F, lambda, F0, ...
  int32_t* istate;    // 8: current edge buffer, candidate valid, accepted, chol failures, pivot failed
};

size_t pgo_workspace_bytes(const PgoPlan& P);
PgoWork pgo_carve(const PgoPlan& P, void* ws);

}  // namespace ba
