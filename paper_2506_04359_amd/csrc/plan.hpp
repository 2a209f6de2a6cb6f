// Host-side plan of a bundle-adjustment window and of a batch of windows.
//
// The plan turns the user's observation index lists (pose i, landmark j,
// camera k per observation, the observed set of Eq. 3 in Sec. 2.2) into the
// landmark-major layout the device kernels stream:
//
//   observations  sorted by (landmark, pose is fixed, free slot / pose, camera)
//   pairs         maximal runs of one (landmark, pose): the W_ij blocks
//   landmarks     contiguous pair ranges, free pairs first
//   tiles         runs of whole landmarks with at most TP pairs: one pass of a
//                 workgroup's per-pair / per-landmark phases
//   chunks        runs of tiles of one window with about `chunk_obs`
//                 observations: one workgroup of the Schur kernels; each chunk
//                 owns a private partial of the reduced camera system
//
// Plain C++ (no HIP) so that it can be built and sanitised on the host alone.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace ba {

constexpr int kMaxPoses = 64;        // poses per window (LDS pose cache)
constexpr int kMaxCams = 32;         // cameras per window (LDS camera cache)
constexpr int kMaxFree = 32;         // free poses per window (6 x 32 = 192 = n_S)
constexpr int kMaxFreeFp64 = 29;     // FP64 partial of S must fit in LDS
constexpr int kMaxObsPerLandmark = 4096;
constexpr int kTileSmall = 64;       // pairs per tile, small-LDS configuration
constexpr int kTileLarge = 256;      // pairs per tile, large configuration
constexpr int kBS = 37;              // stored stride of a 6x6 block (odd: spreads LDS banks)
constexpr int kClasses = 4;          // size classes of chunks (limits below)
// Largest free-pose count of each size class of pass A.  With 256-pair tiles
// and FP32 blocks, windows of up to 23 free poses fit two workgroups per CU.
constexpr int kClassNf[kClasses] = {8, 16, 23, 32};

struct HostWindow {
  int32_t n_poses = 0, n_points = 0, n_cams = 0, n_free = 0;
  int64_t n_obs = 0;
  std::vector<uint8_t> fixed;          // per pose
  std::vector<int32_t> free_slot;      // per pose, -1 when fixed
  std::vector<double> cam;             // per camera: fx fy cx cy R(9) t(3)
  // landmark-major plan order
  std::vector<int32_t> perm;           // plan position -> user observation index
  std::vector<uint8_t> obs_cam;        // plan order
  std::vector<int32_t> pair_obs_begin; // n_pairs + 1, window-local plan positions
  std::vector<int32_t> pair_lm;        // n_pairs, window-local landmark
  std::vector<uint8_t> pair_pose;      // n_pairs, window-local pose
  std::vector<int32_t> lm_pair_begin;  // n_points + 1, window-local pair index
  std::vector<uint8_t> lm_nfree;       // free pairs of each landmark (they come first)
  int64_t schur_blocks = 0;            // sum of P(P+1)/2 over landmarks
  int64_t n_free_pairs = 0;            // sum of P over landmarks
  int64_t n_pairs() const { return (int64_t)pair_pose.size(); }
};

// Validate and build.  Returns an empty string on success, else the error.
// code_out: 0 ok, -1 invalid argument, -5 unsupported structure.
// Camera records (fx fy cx cy, R_cb row-major, t_cb) of a rig after checking
// the intrinsics (finite, fx, fy > 0) and extrinsics (finite, R a rotation;
// NULL: identity).  Returns an error message, empty on success.
std::string pack_cameras(int32_t n_cams, const double* intrinsics, const double* extrinsics,
                         std::vector<double>& cam);

std::string build_window(int32_t n_poses, int32_t n_points, int32_t n_cams, int64_t n_obs,
                         const int32_t* obs_pose, const int32_t* obs_point,
                         const int32_t* obs_cam, const uint8_t* pose_fixed,
                         const double* intrinsics, const double* extrinsics, HostWindow& out,
                         int* code_out);

// Tiles and chunks of a batch for one tile size and chunk target.
struct LaunchTables {
  int tp = 0;                            // pairs per tile
  int chunk_obs = 0;                     // observation target per chunk
  std::vector<int32_t> tile_lm_begin;    // n_tiles + 1, batch-global landmark
  std::vector<int32_t> chunk_window;     // n_chunks
  std::vector<int32_t> chunk_tile_begin; // n_chunks + 1
  std::vector<int32_t> win_chunk_begin;  // n_windows + 1
  std::vector<int64_t> chunk_part_off;   // n_chunks, element offset of its S partial
  std::vector<int32_t> chunk_order;      // n_chunks, grouped by size class
  int32_t class_begin[kClasses + 1] = {0, 0, 0, 0, 0};
  std::vector<int32_t> win_order;        // n_windows, grouped by size class
  int32_t class_win_begin[kClasses + 1] = {0, 0, 0, 0, 0};
  int32_t class_win_nf[kClasses] = {0, 0, 0, 0};   // largest n_free of the class's windows
  int32_t class_nf[kClasses] = {0, 0, 0, 0};   // largest n_free in each class
  int64_t part_elems = 0;                // total partial elements
  // Per tile, the order in which its pairs are handled: free pairs sorted by
  // free slot (so that equal poses sit in adjacent lanes), then fixed pairs.
  // Record of the pair handled by thread t of a tile, at pair_rec[4 (p0 + t)]:
  // {first observation, landmark (both batch-global), pose | q << 8 | nobs << 16,
  //  free slot or -1}; q = the pair's tile-local index in landmark order.
  std::vector<int32_t> pair_rec;         // 4 per pair (batch)
  // Per tile: {first pair, pairs, first landmark, landmarks, first list word,
  // segments, products, 0}, batch-global.
  std::vector<int32_t> tile_rec;         // 8 per tile
  // Per tile, the Schur products (a, b) of pairs of one landmark (a < b,
  // both free; a pair's product with itself is summed per pose instead)
  // grouped by their off-diagonal target block of S: segments of
  // (target block, first product, count), longest first.
  // Stored per tile as one word stream: nseg segment words
  // (blk | start << 10 | len << 23), then the products two per word
  // (qa | qc << 8 as 16-bit halves).
  std::vector<uint32_t> lists;
  int32_t max_tile_prods = 0, max_tile_segs = 0, max_tile_words = 0;
  int32_t n_tiles() const { return (int32_t)tile_lm_begin.size() - 1; }
  int32_t n_chunks() const { return (int32_t)chunk_window.size(); }
};

// Elements of one chunk's partial: the upper 6x6 blocks of S (kBS each), then
// the reduced right-hand side (6 n_free) and diag(U) (6 n_free).
inline int64_t partial_elems(int n_free) {
  const int64_t nblk = (int64_t)n_free * (n_free + 1) / 2;
  return nblk * kBS + 12 * (int64_t)n_free;
}

inline int size_class(int n_free) {
  for (int c = 0; c < kClasses; ++c)
    if (n_free <= kClassNf[c]) return c;
  return kClasses - 1;
}

// Tiles, product lists and work items of a launch: tiles of at most tp pairs,
// work items of about chunk_obs x class_mult[size class] observations
// (class_mult NULL: 1 for every class).
void build_tiles(const std::vector<const HostWindow*>& wins, int tp, int chunk_obs,
                 LaunchTables& out, const int* class_mult = nullptr);

// Packed fields of the plan tables and the limits that keep them in range.
//   segment word : blk (10 bits) | first product (13 bits) | count (9 bits)
//   product      : qa (8 bits) | qc (8 bits), tile-local pair indices
//   pair record  : pose (8 bits) | q (8 bits) | observations of the pair (15 bits)
constexpr int kSegBlkBits = 10, kSegStartBits = 13, kSegLenBits = 9;
static_assert(kSegBlkBits + kSegStartBits + kSegLenBits == 32, "segment word is 32 bits");
// target blocks of S: nf (nf + 1) / 2 upper blocks
static_assert(kMaxFree * (kMaxFree + 1) / 2 <= (1 << kSegBlkBits), "block index field too narrow");
// products of one tile: sum over its landmarks of P (P - 1) / 2 with sum P <= TP
// and P <= kMaxFree, at most TP (kMaxFree - 1) / 2
static_assert(kTileLarge * (kMaxFree - 1) / 2 < (1 << kSegStartBits), "product index field too narrow");
// products of one target block in one tile: one per landmark, at most TP / 2
static_assert(kTileLarge / 2 < (1 << kSegLenBits), "product count field too narrow");
static_assert(kTileSmall <= kTileLarge && kTileLarge <= 256, "tile-local pair index is 8 bits");
static_assert(kMaxPoses <= 256, "pose index of a pair record is 8 bits");
static_assert(kMaxObsPerLandmark < (1 << 15), "observations of a pair record are 15 bits");

// Segment word of the product lists.
inline uint32_t seg_word(int blk, int start, int len) {
  return (uint32_t)blk | ((uint32_t)start << kSegBlkBits) |
         ((uint32_t)len << (kSegBlkBits + kSegStartBits));
}

}  // namespace ba
