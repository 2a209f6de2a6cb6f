// Host check of the plan builders (window plan, launch tables, pose-graph
// plan) on seeded random structures, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_plan_sanitize.py.  Every packed
// field of the launch tables is decoded and checked against the structure it
// came from; any violation prints a message and exits non-zero, any memory or
// UB error aborts through the sanitizers.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "../../paper_2506_04359_amd/csrc/pgo_plan.hpp"
#include "../../paper_2506_04359_amd/csrc/plan.hpp"

using namespace ba;

static int g_fail = 0;
#define CHECK(c, ...)                                   \
  do {                                                  \
    if (!(c)) {                                         \
      std::fprintf(stderr, "check failed: %s: ", #c);   \
      std::fprintf(stderr, __VA_ARGS__);                \
      std::fprintf(stderr, "\n");                       \
      if (++g_fail > 20) std::exit(1);                  \
    }                                                   \
  } while (0)

struct Obs {
  std::vector<int32_t> pose, point, cam;
};

// Random window: landmarks seen from 2..track distinct (pose, camera) views,
// some poses fixed, several cameras.
static Obs random_window(std::mt19937& rng, int n_poses, int n_points, int n_cams, int max_track) {
  Obs o;
  std::uniform_int_distribution<int> up(0, n_poses - 1), uc(0, n_cams - 1);
  std::uniform_int_distribution<int> ut(2, max_track);
  for (int j = 0; j < n_points; ++j) {
    const int t = ut(rng);
    std::set<std::pair<int, int>> views;
    while ((int)views.size() < std::min(t, n_poses * n_cams)) views.insert({up(rng), uc(rng)});
    for (auto& v : views) {
      const int reps = (rng() % 7 == 0) ? 2 : 1;   // repeated observations of one view
      for (int r = 0; r < reps; ++r) {
        o.pose.push_back(v.first);
        o.point.push_back(j);
        o.cam.push_back(v.second);
      }
    }
  }
  // user order shuffled
  std::vector<int> idx(o.pose.size());
  for (size_t k = 0; k < idx.size(); ++k) idx[k] = (int)k;
  std::shuffle(idx.begin(), idx.end(), rng);
  Obs s;
  for (int k : idx) {
    s.pose.push_back(o.pose[k]);
    s.point.push_back(o.point[k]);
    s.cam.push_back(o.cam[k]);
  }
  return s;
}

static void check_window(const HostWindow& w, const Obs& o) {
  const int64_t n = w.n_obs;
  CHECK((int64_t)w.perm.size() == n, "perm size");
  std::vector<char> seen(n, 0);
  for (int64_t k = 0; k < n; ++k) {
    CHECK(w.perm[k] >= 0 && w.perm[k] < n, "perm range");
    if (w.perm[k] >= 0 && w.perm[k] < n) seen[w.perm[k]]++;
  }
  for (int64_t k = 0; k < n; ++k) CHECK(seen[k] == 1, "perm is a permutation");
  CHECK((int64_t)w.pair_obs_begin.size() == w.n_pairs() + 1, "pair_obs_begin size");
  for (int64_t q = 0; q < w.n_pairs(); ++q) {
    const int32_t a = w.pair_obs_begin[q], b = w.pair_obs_begin[q + 1];
    CHECK(a < b, "pair has observations");
    for (int32_t k = a; k < b; ++k) {
      CHECK(o.point[w.perm[k]] == w.pair_lm[q], "pair landmark");
      CHECK(o.pose[w.perm[k]] == w.pair_pose[q], "pair pose");
    }
  }
  for (int j = 0; j < w.n_points; ++j) {
    const int32_t a = w.lm_pair_begin[j], b = w.lm_pair_begin[j + 1];
    int nfree = 0;
    bool fixed_seen = false;
    for (int32_t q = a; q < b; ++q) {
      CHECK(w.pair_lm[q] == j, "landmark pair range");
      const bool fx = w.fixed[w.pair_pose[q]] != 0;
      if (!fx) {
        CHECK(!fixed_seen, "free pairs come first");
        ++nfree;
      } else {
        fixed_seen = true;
      }
    }
    CHECK(nfree == w.lm_nfree[j], "free pair count");
  }
}

static void check_tables(const HostWindow& w, const LaunchTables& t) {
  const int tp = t.tp;
  const int nblk = w.n_free * (w.n_free + 1) / 2;
  CHECK(t.n_tiles() >= (w.n_points > 0 ? 1 : 0), "tiles");
  std::vector<int> pair_seen(w.n_pairs(), 0);
  for (int ti = 0; ti < t.n_tiles(); ++ti) {
    const int32_t* rec = &t.tile_rec[8 * ti];
    const int p0 = rec[0], np = rec[1], l0 = rec[2], nl = rec[3], w0 = rec[4], nseg = rec[5], nprod = rec[6];
    CHECK(np >= 1 && np <= tp, "tile pairs %d", np);
    CHECK(nl >= 1 && nl <= tp / 2, "tile landmarks %d", nl);
    CHECK(l0 == t.tile_lm_begin[ti] && l0 + nl == t.tile_lm_begin[ti + 1], "tile landmark range");
    CHECK(p0 == w.lm_pair_begin[l0] && p0 + np == w.lm_pair_begin[l0 + nl], "tile pair range");
    // pair records: every pair of the tile once, free ones sorted by slot
    int prev_slot = -1;
    bool fixed_seen = false;
    for (int th = 0; th < np; ++th) {
      const int32_t* pr = &t.pair_rec[4 * (p0 + th)];
      const int pose = pr[2] & 255, q = (pr[2] >> 8) & 255, nobs = pr[2] >> 16;
      CHECK(q >= 0 && q < np, "pair q %d", q);
      const int wp = p0 + q;
      if (wp < 0 || wp >= w.n_pairs()) continue;
      pair_seen[wp]++;
      CHECK(pr[0] == w.pair_obs_begin[wp], "pair first observation");
      CHECK(pr[1] == w.pair_lm[wp], "pair landmark");
      CHECK(pose == w.pair_pose[wp], "pair pose");
      CHECK(nobs == w.pair_obs_begin[wp + 1] - w.pair_obs_begin[wp], "pair observations");
      CHECK(pr[3] == w.free_slot[pose], "pair slot");
      if (pr[3] >= 0) {
        CHECK(!fixed_seen && pr[3] >= prev_slot, "free pairs by slot");
        prev_slot = pr[3];
      } else {
        fixed_seen = true;
      }
    }
    // product lists: segments cover the products, every product is a pair of
    // free pairs of one landmark whose slots name the target block
    CHECK(w0 >= 0 && w0 + nseg + (nprod + 1) / 2 <= (int)t.lists.size(), "list words in range");
    if (w0 < 0 || w0 + nseg + (nprod + 1) / 2 > (int)t.lists.size()) continue;
    int covered = 0;
    for (int s = 0; s < nseg; ++s) {
      const uint32_t wd = t.lists[w0 + s];
      const int blk = wd & ((1u << kSegBlkBits) - 1);
      const int start = (wd >> kSegBlkBits) & ((1u << kSegStartBits) - 1);
      const int len = wd >> (kSegBlkBits + kSegStartBits);
      CHECK(blk < nblk, "segment block");
      CHECK(start == covered && len >= 1, "segments contiguous");
      covered = start + len;
      for (int k = start; k < start + len && k < nprod; ++k) {
        const uint32_t word = t.lists[w0 + nseg + k / 2];
        const uint32_t pp = (k & 1) ? (word >> 16) : (word & 0xffff);
        const int qa = pp & 255, qc = pp >> 8;
        CHECK(qa < qc && qc < np, "product pairs ordered and in the tile");
        if (!(qa < qc && qc < np)) continue;
        CHECK(w.pair_lm[p0 + qa] == w.pair_lm[p0 + qc], "product pairs share a landmark");
        const int sa = w.free_slot[w.pair_pose[p0 + qa]], sb = w.free_slot[w.pair_pose[p0 + qc]];
        CHECK(sa >= 0 && sb >= 0 && sa < sb, "product pairs free, slots ordered");
        const int want = sa * w.n_free - (sa * (sa - 1)) / 2 + (sb - sa);
        CHECK(want == blk, "product target block");
      }
    }
    CHECK(covered == nprod, "segments cover every product");
    int expect = 0;
    for (int l = l0; l < l0 + nl; ++l) expect += w.lm_nfree[l] * (w.lm_nfree[l] - 1) / 2;
    CHECK(expect == nprod, "product count");
  }
  for (int64_t q = 0; q < w.n_pairs(); ++q) CHECK(pair_seen[q] == 1, "pair in one tile once");
  // chunks: contiguous tile ranges of the window, partial offsets disjoint
  CHECK(t.n_chunks() >= 1, "a window has a chunk");
  for (int c = 0; c < t.n_chunks(); ++c) {
    CHECK(t.chunk_tile_begin[c] <= t.chunk_tile_begin[c + 1], "chunk tile range");
    CHECK(t.chunk_part_off[c] == c * partial_elems(w.n_free), "partial offset");
  }
  CHECK(t.chunk_tile_begin[t.n_chunks()] == t.n_tiles(), "chunks cover the tiles");
  std::vector<char> in_order(t.n_chunks(), 0);
  for (int k : t.chunk_order) {
    CHECK(k >= 0 && k < t.n_chunks(), "chunk order range");
    if (k >= 0 && k < t.n_chunks()) in_order[k]++;
  }
  for (int c = 0; c < t.n_chunks(); ++c) CHECK(in_order[c] == 1, "chunk order is a permutation");
}

static void check_pgo(const PgoPlan& P) {
  const int nf = P.n_free, nb = P.n_blocks();
  CHECK((int)P.blk_ptr.size() == nf + 1, "blk_ptr");
  for (int c = 0; c < nf; ++c) {
    CHECK(P.blk_row[P.blk_ptr[c]] == c, "diagonal block first");
    for (int b = P.blk_ptr[c] + 1; b < P.blk_ptr[c + 1]; ++b)
      CHECK(P.blk_row[b] > P.blk_row[b - 1] && P.blk_row[b] < nf, "rows increase");
  }
  CHECK((int)P.upd_ptr.size() == nb + 1 && P.upd_a.size() == P.upd_b.size(), "update lists");
  for (size_t k = 0; k < P.upd_a.size(); ++k)
    CHECK(P.upd_a[k] >= 0 && P.upd_a[k] < nb && P.upd_b[k] >= 0 && P.upd_b[k] < nb, "update block ids");
  for (int b = 0; b < nb; ++b)
    for (int k = P.upd_ptr[b]; k < P.upd_ptr[b + 1]; ++k) {
      // L_ra L_cb^T with both from one column k < target column, rows r, c
      const int a = P.upd_a[k], bb = P.upd_b[k];
      CHECK(P.blk_col[a] == P.blk_col[bb], "update factors of one column");
      CHECK(P.blk_row[a] == P.blk_row[b] && P.blk_row[bb] == P.blk_col[b], "update target");
      CHECK(P.blk_col[a] < P.blk_col[b], "update from an earlier column");
    }
  for (size_t k = 0; k < P.fwd_blk.size(); ++k)
    CHECK(P.fwd_blk[k] >= 0 && P.fwd_blk[k] < nb && P.fwd_col[k] >= 0 && P.fwd_col[k] < nf, "forward ids");
  for (size_t k = 0; k < P.asm_edge.size(); ++k)
    CHECK(P.asm_edge[k] >= 0 && P.asm_edge[k] < 2 * P.n_edges, "assembly edges");
  for (size_t k = 0; k < P.rhs_edge.size(); ++k)
    CHECK(P.rhs_edge[k] >= 0 && P.rhs_edge[k] < 2 * P.n_edges, "rhs edges");
  CHECK((int)P.lev_ptr.size() == P.n_levels + 1 && (nf == 0 || P.lev_ptr[P.n_levels] == nf), "levels");
  for (size_t q = 0; q < P.chunk_blk.size(); ++q) CHECK(P.chunk_blk[q] >= 0 && P.chunk_blk[q] < nb, "chunk block");
  for (size_t q = 0; q < P.fchunk_col.size(); ++q) CHECK(P.fchunk_col[q] >= 0 && P.fchunk_col[q] < nf, "chunk col");
}

int main(int argc, char** argv) {
  const int rounds = argc > 1 ? std::atoi(argv[1]) : 60;
  std::mt19937 rng(12345);
  int windows = 0, graphs = 0, rejects = 0;
  for (int r = 0; r < rounds; ++r) {
    const int n_poses = 1 + (int)(rng() % kMaxPoses);
    const int n_cams = 1 + (int)(rng() % 4);
    const int n_points = (int)(rng() % 400);
    const int max_track = 2 + (int)(rng() % 12);
    Obs o = random_window(rng, n_poses, n_points, n_cams, max_track);
    std::vector<uint8_t> fixed(n_poses, 0);
    // free poses up to the limit, a few beyond it to reach the error path
    const int want_free = (int)(rng() % (kMaxFree + 4));
    for (int i = 0; i < n_poses; ++i) fixed[i] = i >= want_free;
    if (n_poses > 0 && rng() % 3 == 0) fixed[0] = 1;
    std::vector<double> K(4 * n_cams), E(12 * n_cams, 0.0);
    for (int k = 0; k < n_cams; ++k) {
      K[4 * k] = K[4 * k + 1] = 400.0 + k;
      K[4 * k + 2] = 320.0;
      K[4 * k + 3] = 240.0;
      E[12 * k] = E[12 * k + 5] = E[12 * k + 10] = 1.0;
      E[12 * k + 3] = 0.1 * k;
    }
    // occasionally corrupt one index to exercise the validation
    if (!o.pose.empty() && rng() % 5 == 0) o.pose[rng() % o.pose.size()] = n_poses + (int)(rng() % 3);
    HostWindow w;
    int code = 0;
    const std::string err = build_window(n_poses, n_points, n_cams, (int64_t)o.pose.size(), o.pose.data(),
                                         o.point.data(), o.cam.data(), fixed.data(), K.data(), E.data(), w, &code);
    if (code != 0) {
      CHECK(!err.empty(), "an error carries a message");
      ++rejects;
      continue;
    }
    ++windows;
    check_window(w, o);
    for (int tp : {kTileSmall, kTileLarge})
      for (int chunk : {512, 2048, 16384}) {
        LaunchTables t;
        build_tiles({&w}, tp, chunk, t);
        check_tables(w, t);
      }
  }
  // a batch of several windows in one table
  {
    std::vector<HostWindow> ws;
    for (int k = 0; k < 6; ++k) {
      const int n_poses = 5 + 5 * k;
      Obs o = random_window(rng, n_poses, 300 + 50 * k, 1, 8);
      std::vector<uint8_t> fixed(n_poses, 0);
      fixed[0] = 1;
      const double K[4] = {458, 458, 367, 248};
      HostWindow w;
      int code = 0;
      build_window(n_poses, 300 + 50 * k, 1, (int64_t)o.pose.size(), o.pose.data(), o.point.data(), nullptr,
                   fixed.data(), K, nullptr, w, &code);
      CHECK(code == 0, "batch window builds");
      ws.push_back(w);
    }
    std::vector<const HostWindow*> ptrs;
    for (auto& w : ws) ptrs.push_back(&w);
    LaunchTables t;
    build_tiles(ptrs, kTileLarge, 1024, t);
    CHECK((int)t.win_chunk_begin.size() == 7, "window chunk ranges");
    for (int c = 0; c < kClasses; ++c) CHECK(t.class_begin[c] <= t.class_begin[c + 1], "class ranges");
  }
  for (int r = 0; r < rounds; ++r) {
    const int n = 1 + (int)(rng() % 300);
    std::vector<int32_t> ei, ej;
    for (int i = 1; i < n; ++i) {   // a chain plus random chords
      ei.push_back(i - 1);
      ej.push_back(i);
    }
    const int extra = (int)(rng() % (2 * n + 1));
    for (int k = 0; k < extra; ++k) {
      const int a = (int)(rng() % n), b = (int)(rng() % n);
      if (a != b) {
        ei.push_back(a);
        ej.push_back(b);
      }
    }
    std::vector<uint8_t> fixed(n, 0);
    fixed[rng() % n] = 1;
    if (rng() % 4 == 0 && !ei.empty()) {   // a self-loop: rejected
      const size_t k = rng() % ej.size();
      ej[k] = ei[k];
    }
    PgoPlan P;
    const std::string err = build_pgo_plan(n, (int32_t)ei.size(), ei.data(), ej.data(), fixed.data(), P);
    if (!err.empty()) {
      ++rejects;
      continue;
    }
    ++graphs;
    check_pgo(P);
    CHECK(pgo_workspace_bytes(P) > 0, "workspace");
  }
  std::printf("plan_check: %d windows, %d graphs, %d rejected inputs, %d failures\n", windows, graphs, rejects,
              g_fail);
  return g_fail ? 1 : 0;
}
