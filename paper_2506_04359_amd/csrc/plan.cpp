// Host-side plan construction (see plan.hpp).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <sstream>

namespace ba {

namespace {

std::string fail(int* code, int c, const std::string& msg) {
  *code = c;
  return msg;
}

bool rotation_ok(const double* R) {
  // R R^T = I within 1e-6 and det > 0
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      double s = 0;
      for (int c = 0; c < 3; ++c) s += R[3 * a + c] * R[3 * b + c];
      if (std::fabs(s - (a == b ? 1.0 : 0.0)) > 1e-6) return false;
    }
  const double det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                     R[2] * (R[3] * R[7] - R[4] * R[6]);
  return det > 0;
}

}  // namespace

std::string pack_cameras(int32_t n_cams, const double* intrinsics, const double* extrinsics,
                         std::vector<double>& cam) {
  cam.assign((size_t)n_cams * 16, 0.0);
  for (int k = 0; k < n_cams; ++k) {
    const double* K = intrinsics + 4 * k;
    for (int c = 0; c < 4; ++c)
      if (!std::isfinite(K[c])) return "non-finite intrinsics";
    if (!(K[0] > 0 && K[1] > 0)) return "focal lengths must be positive";
    double* C = cam.data() + 16 * k;
    for (int c = 0; c < 4; ++c) C[c] = K[c];
    if (extrinsics) {
      const double* E = extrinsics + 12 * k;
      for (int c = 0; c < 12; ++c)
        if (!std::isfinite(E[c])) return "non-finite extrinsics";
      const double R[9] = {E[0], E[1], E[2], E[4], E[5], E[6], E[8], E[9], E[10]};
      if (!rotation_ok(R)) return "extrinsic rotation is not a rotation";
      for (int c = 0; c < 9; ++c) C[4 + c] = R[c];
      C[13] = E[3];
      C[14] = E[7];
      C[15] = E[11];
    } else {
      C[4] = C[8] = C[12] = 1.0;
    }
  }
  return "";
}

std::string build_window(int32_t n_poses, int32_t n_points, int32_t n_cams, int64_t n_obs,
                         const int32_t* obs_pose, const int32_t* obs_point,
                         const int32_t* obs_cam, const uint8_t* pose_fixed,
                         const double* intrinsics, const double* extrinsics, HostWindow& w,
                         int* code) {
  *code = 0;
  if (n_poses < 1) return fail(code, -1, "n_poses must be >= 1");
  if (n_points < 0 || n_cams < 1 || n_obs < 0) return fail(code, -1, "negative size");
  if (n_obs > 0 && (!obs_pose || !obs_point)) return fail(code, -1, "obs_pose/obs_point is NULL");
  if (!intrinsics) return fail(code, -1, "intrinsics is NULL");
  if (n_poses > kMaxPoses) return fail(code, -5, "more than 64 poses in a window");
  if (n_cams > kMaxCams) return fail(code, -5, "more than 32 cameras in a window");
  if (n_obs > (int64_t)INT32_MAX / 2) return fail(code, -5, "too many observations");

  w.n_poses = n_poses;
  w.n_points = n_points;
  w.n_cams = n_cams;
  w.n_obs = n_obs;
  w.fixed.assign(n_poses, 0);
  if (pose_fixed) {
    for (int i = 0; i < n_poses; ++i) w.fixed[i] = pose_fixed[i] ? 1 : 0;
  } else {
    w.fixed[0] = 1;
  }
  w.free_slot.assign(n_poses, -1);
  w.n_free = 0;
  for (int i = 0; i < n_poses; ++i)
    if (!w.fixed[i]) w.free_slot[i] = w.n_free++;
  if (w.n_free > kMaxFree) return fail(code, -5, "more than 32 free poses in a window");

  {
    const std::string m = pack_cameras(n_cams, intrinsics, extrinsics, w.cam);
    if (!m.empty()) return fail(code, -1, m);
  }

  for (int64_t o = 0; o < n_obs; ++o) {
    if (obs_pose[o] < 0 || obs_pose[o] >= n_poses) {
      std::ostringstream s;
      s << "obs_pose[" << o << "] = " << obs_pose[o] << " out of range";
      return fail(code, -1, s.str());
    }
    if (obs_point[o] < 0 || obs_point[o] >= n_points) {
      std::ostringstream s;
      s << "obs_point[" << o << "] = " << obs_point[o] << " out of range";
      return fail(code, -1, s.str());
    }
    if (obs_cam && (obs_cam[o] < 0 || obs_cam[o] >= n_cams)) {
      std::ostringstream s;
      s << "obs_cam[" << o << "] = " << obs_cam[o] << " out of range";
      return fail(code, -1, s.str());
    }
  }

  // landmark-major order: (landmark, fixed, free slot or pose, camera, user
  // index).  Each observation gets a 64-bit key (pose key, camera, user
  // index) in one sequential pass; a stable counting sort by landmark puts
  // the keys in landmark runs (user order inside a run), and each run, short
  // and contiguous, is sorted by key.  Everything after reads the sorted keys
  // in order.
  auto cam_of = [&](int64_t o) { return obs_cam ? obs_cam[o] : 0; };
  int32_t pose_of_key[2 * kMaxPoses];
  auto pose_key = [&](int32_t i) {
    return w.fixed[i] ? (int32_t)(kMaxPoses + i) : w.free_slot[i];
  };
  for (int i = 0; i < n_poses; ++i) pose_of_key[pose_key(i)] = i;
  std::vector<int64_t> start((size_t)n_points + 1, 0);
  std::vector<uint64_t> key(n_obs);
  {
    for (int64_t o = 0; o < n_obs; ++o) start[obs_point[o] + 1]++;
    for (int32_t j = 0; j < n_points; ++j) start[j + 1] += start[j];
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t o = 0; o < n_obs; ++o) {
      const uint64_t k = ((uint64_t)pose_key(obs_pose[o]) << 40) | ((uint64_t)cam_of(o) << 32) | (uint64_t)o;
      key[fill[obs_point[o]]++] = k;
    }
    for (int32_t j = 0; j < n_points; ++j) {
      uint64_t* b = key.data() + start[j];
      const int64_t len = start[j + 1] - start[j];
      if (len <= 32) {
        for (int64_t x = 1; x < len; ++x) {   // insertion sort
          const uint64_t v = b[x];
          int64_t y = x;
          for (; y > 0 && v < b[y - 1]; --y) b[y] = b[y - 1];
          b[y] = v;
        }
      } else {
        std::sort(b, b + len);
      }
    }
  }
  w.perm.resize(n_obs);
  w.obs_cam.resize(n_obs);
  for (int64_t k = 0; k < n_obs; ++k) {
    w.perm[k] = (int32_t)(key[k] & 0xffffffffu);
    w.obs_cam[k] = (uint8_t)((key[k] >> 32) & 0xff);
  }

  // pairs and landmark ranges
  w.pair_obs_begin.clear();
  w.pair_lm.clear();
  w.pair_pose.clear();
  w.pair_obs_begin.reserve((size_t)n_obs + 1);
  w.pair_lm.reserve((size_t)n_obs);
  w.pair_pose.reserve((size_t)n_obs);
  w.lm_pair_begin.assign((size_t)n_points + 1, 0);
  w.lm_nfree.assign(n_points, 0);
  for (int32_t j = 0; j < n_points; ++j) {
    int views = 0;
    for (int64_t k = start[j]; k < start[j + 1]; ++k) {
      const uint32_t pk = (uint32_t)(key[k] >> 40), cm = (uint32_t)(key[k] >> 32) & 0xff;
      const bool new_pair = k == start[j] || (uint32_t)(key[k - 1] >> 40) != pk;
      const bool new_view = new_pair || ((uint32_t)(key[k - 1] >> 32) & 0xff) != cm;
      if (new_pair) {
        const int32_t i = pose_of_key[pk];
        w.pair_obs_begin.push_back((int32_t)k);
        w.pair_lm.push_back(j);
        w.pair_pose.push_back((uint8_t)i);
        w.lm_pair_begin[j + 1]++;
        if (!w.fixed[i]) w.lm_nfree[j]++;
      }
      if (new_view) views++;
    }
    if (views < 2) {
      std::ostringstream s;
      s << "landmark " << j << " has fewer than 2 distinct (pose, camera) views";
      return fail(code, -1, s.str());
    }
    if (start[j + 1] - start[j] > kMaxObsPerLandmark)
      return fail(code, -5, "too many observations of one landmark");
    w.lm_pair_begin[j + 1] += w.lm_pair_begin[j];
  }
  w.pair_obs_begin.push_back((int32_t)n_obs);
  w.schur_blocks = 0;
  w.n_free_pairs = 0;
  for (int j = 0; j < n_points; ++j) {
    const int64_t P = w.lm_nfree[j];
    w.schur_blocks += P * (P + 1) / 2;
    w.n_free_pairs += P;
  }
  return std::string();
}

void build_tiles(const std::vector<const HostWindow*>& wins, int tp, int chunk_obs,
                 LaunchTables& t, const int* class_mult) {
  t.tp = tp;
  t.chunk_obs = chunk_obs;
  t.tile_lm_begin.clear();
  t.chunk_window.clear();
  t.chunk_tile_begin.clear();
  t.win_chunk_begin.clear();
  t.chunk_part_off.clear();
  t.part_elems = 0;
  t.pair_rec.clear();
  t.tile_rec.clear();
  t.lists.clear();
  t.max_tile_prods = t.max_tile_segs = t.max_tile_words = 0;
  int32_t lm_base = 0, pair_base = 0, obs_base = 0;
  for (size_t wi = 0; wi < wins.size(); ++wi) {
    const HostWindow& w = *wins[wi];
    // tiles: whole landmarks, at most tp pairs and tp / 2 landmarks
    std::vector<int32_t> tiles;      // window-local landmark starts
    std::vector<int64_t> tile_obs;   // observations per tile
    int32_t j = 0;
    while (j < w.n_points) {
      const int32_t start = j;
      int32_t pairs = 0;
      while (j < w.n_points) {
        const int32_t pj = w.lm_pair_begin[j + 1] - w.lm_pair_begin[j];
        if (j > start && (pairs + pj > tp || j - start >= tp / 2)) break;
        pairs += pj;
        ++j;
      }
      tiles.push_back(start);
      const int32_t p0 = w.lm_pair_begin[start], p1 = w.lm_pair_begin[j];
      tile_obs.push_back((int64_t)w.pair_obs_begin[p1] - w.pair_obs_begin[p0]);
    }
    const int32_t first_tile = (int32_t)t.tile_lm_begin.size();
    for (int32_t s : tiles) t.tile_lm_begin.push_back(lm_base + s);
    // per-tile pair order and Schur product lists, by counting sorts (keys
    // are small: free slots, target blocks, product counts)
    const int nblk = w.n_free * (w.n_free + 1) / 2;
    std::vector<int32_t> blk_count(nblk), blk_fill(nblk), ord, slot_start(kMaxFree + 3);
    std::vector<uint16_t> prod_blk_q, prods;   // products in landmark order, then grouped
    std::vector<int32_t> prod_blk;
    std::vector<int32_t> order, size_start(kTileLarge / 2 + 2);
    for (size_t ti = 0; ti < tiles.size(); ++ti) {
      const int32_t la = tiles[ti];
      const int32_t lb = ti + 1 < tiles.size() ? tiles[ti + 1] : w.n_points;
      const int32_t p0 = w.lm_pair_begin[la], p1 = w.lm_pair_begin[lb];
      // pairs stably by free slot (fixed pairs last)
      auto key = [&](int32_t q) {
        const int sl = w.free_slot[w.pair_pose[p0 + q]];
        return sl >= 0 ? sl : kMaxFree + 1;
      };
      std::fill(slot_start.begin(), slot_start.end(), 0);
      for (int32_t q = 0; q < p1 - p0; ++q) slot_start[key(q) + 1]++;
      for (int k = 0; k + 1 < (int)slot_start.size(); ++k) slot_start[k + 1] += slot_start[k];
      ord.resize(p1 - p0);
      for (int32_t q = 0; q < p1 - p0; ++q) ord[slot_start[key(q)]++] = q;
      for (int32_t q : ord) {
        const int32_t wp = p0 + q;   // window-local pair
        const int32_t nobs = w.pair_obs_begin[wp + 1] - w.pair_obs_begin[wp];
        t.pair_rec.push_back(obs_base + w.pair_obs_begin[wp]);
        t.pair_rec.push_back(lm_base + w.pair_lm[wp]);
        t.pair_rec.push_back((int32_t)w.pair_pose[wp] | (q << 8) | (nobs << 16));
        t.pair_rec.push_back(w.free_slot[w.pair_pose[wp]]);
      }
      // products (a, b), a < b, of each landmark's free pairs, with their
      // target block; (a, a) is summed per pair in the kernels
      prod_blk_q.clear();
      prod_blk.clear();
      std::fill(blk_count.begin(), blk_count.end(), 0);
      for (int32_t l = la; l < lb; ++l) {
        const int32_t q0 = w.lm_pair_begin[l] - p0;
        const int nfp = w.lm_nfree[l];
        for (int a = 0; a < nfp; ++a)
          for (int b = a + 1; b < nfp; ++b) {
            const int sa = w.free_slot[w.pair_pose[p0 + q0 + a]];
            const int sb = w.free_slot[w.pair_pose[p0 + q0 + b]];
            const int blk = sa * w.n_free - (sa * (sa - 1)) / 2 + (sb - sa);
            prod_blk_q.push_back((uint16_t)((q0 + a) | ((q0 + b) << 8)));
            prod_blk.push_back(blk);
            blk_count[blk]++;
          }
      }
      // target blocks by product count, largest first, ties in block order
      std::fill(size_start.begin(), size_start.end(), 0);
      int nseg = 0;
      for (int k = 0; k < nblk; ++k)
        if (blk_count[k] > 0) {
          size_start[kTileLarge / 2 + 1 - blk_count[k]]++;
          ++nseg;
        }
      for (int k = 0; k + 1 < (int)size_start.size(); ++k) size_start[k + 1] += size_start[k];
      order.resize(nseg);
      for (int k = 0; k < nblk; ++k)
        if (blk_count[k] > 0) order[size_start[kTileLarge / 2 - blk_count[k]]++] = k;
      const int32_t word_first = (int32_t)t.lists.size();
      int start = 0;
      for (int k : order) {
        t.lists.push_back(seg_word(k, start, blk_count[k]));
        blk_fill[k] = start;
        start += blk_count[k];
      }
      prods.resize(start);
      for (size_t x = 0; x < prod_blk.size(); ++x) prods[blk_fill[prod_blk[x]]++] = prod_blk_q[x];
      for (size_t k = 0; k < prods.size(); k += 2)
        t.lists.push_back((uint32_t)prods[k] | ((k + 1 < prods.size() ? (uint32_t)prods[k + 1] : 0u) << 16));
      t.max_tile_prods = std::max(t.max_tile_prods, start);
      t.max_tile_segs = std::max(t.max_tile_segs, (int32_t)order.size());
      t.max_tile_words = std::max(t.max_tile_words, (int32_t)t.lists.size() - word_first);
      const int32_t rec[8] = {pair_base + p0, p1 - p0, lm_base + la, lb - la,
                              word_first, (int32_t)order.size(), start, 0};
      t.tile_rec.insert(t.tile_rec.end(), rec, rec + 8);
    }
    // chunks: split the window's tiles into about n_obs / chunk_obs runs of
    // balanced observation counts; a window always has at least one chunk
    t.win_chunk_begin.push_back((int32_t)t.chunk_window.size());
    const int64_t nt = (int64_t)tiles.size();
    const int64_t co = (int64_t)chunk_obs * (class_mult ? class_mult[size_class(w.n_free)] : 1);
    int64_t want = std::max<int64_t>(1, (w.n_obs + co / 2) / std::max<int64_t>(1, co));
    want = std::min<int64_t>(want, std::max<int64_t>(1, nt));
    int64_t done_obs = 0, k = 0;
    const int64_t pe = partial_elems(w.n_free);
    for (int64_t c = 0; c < want; ++c) {
      t.chunk_window.push_back((int32_t)wi);
      t.chunk_tile_begin.push_back(first_tile + (int32_t)k);
      t.chunk_part_off.push_back(t.part_elems);
      t.part_elems += pe;
      // advance until this chunk holds its share of the remaining observations
      const int64_t target = (w.n_obs * (c + 1)) / want;
      const int64_t left = want - c - 1;          // chunks still to place
      while (k < nt && (done_obs < target || k == (int64_t)t.chunk_tile_begin.back() - first_tile) &&
             nt - k > left) {
        done_obs += tile_obs[k];
        ++k;
      }
    }
    lm_base += w.n_points;
    pair_base += (int32_t)w.n_pairs();
    obs_base += (int32_t)w.n_obs;
  }
  t.lists.push_back(0u);   // padding: the kernels read a tile's words unconditionally, clamped to its last
  t.tile_lm_begin.push_back(lm_base);
  t.chunk_tile_begin.push_back((int32_t)t.tile_lm_begin.size() - 1);
  t.win_chunk_begin.push_back((int32_t)t.chunk_window.size());
  // group chunks by size class (stable: windows stay in order inside a class)
  t.chunk_order.clear();
  for (int c = 0; c < kClasses; ++c) {
    t.class_begin[c] = (int32_t)t.chunk_order.size();
    t.class_nf[c] = 0;
    for (int32_t k = 0; k < t.n_chunks(); ++k) {
      const int nf = wins[t.chunk_window[k]]->n_free;
      if (size_class(nf) == c) {
        t.chunk_order.push_back(k);
        t.class_nf[c] = std::max(t.class_nf[c], nf);
      }
    }
  }
  t.class_begin[kClasses] = (int32_t)t.chunk_order.size();
  // the windows of each class, in window order (every chunk of a window is in
  // its window's class)
  t.win_order.clear();
  for (int c = 0; c < kClasses; ++c) {
    t.class_win_begin[c] = (int32_t)t.win_order.size();
    t.class_win_nf[c] = 0;
    for (int32_t i = 0; i < (int32_t)wins.size(); ++i)
      if (size_class(wins[i]->n_free) == c) {
        t.win_order.push_back(i);
        t.class_win_nf[c] = std::max(t.class_win_nf[c], wins[i]->n_free);
      }
  }
  t.class_win_begin[kClasses] = (int32_t)t.win_order.size();
}

}  // namespace ba
