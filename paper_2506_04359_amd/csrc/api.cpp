// C ABI of the bundle adjuster (include/ba.h): argument checks, plan upload,
// workspace layout, launch-shape selection and the launch sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <memory>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/ba.h"
#include "device.hpp"
#include "plan.hpp"
#include "pnp.hpp"
#include "tri.hpp"
#include "pgo.hpp"
#include "vi.hpp"

// Device scratch of ba_solve_noalloc: one copy per GPU the library runs on,
// held until the process ends.  Host code never passes this name to a kernel
// or a copy (on the host it is only a stand-in for the symbol): it uses the
// per-device address that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[BA_NOALLOC_SCRATCH_BYTES];

namespace ba {

// defined in kernels.hip
template <typename Real, int TP>
size_t pass_a_lds(int np, int nc, int nf, int list_bytes, bool adj);
template <typename Real, int TP>
size_t pass_b_lds();
size_t reduce_lds(int max_nf);
template <typename Real, int TP, bool ADJ>
hipError_t set_attrs();
template <typename Real, int TP>
hipError_t run_solve(const LaunchArgs& A, const DevWork<Real>& K);
template <typename Real, int TP>
hipError_t run_adjoint(const LaunchArgs& A, const DevWork<Real>& K);
template <typename Real, int TP>
hipError_t run_solve_timed(const LaunchArgs& A, const DevWork<Real>& K, double* stage_ms);

constexpr size_t kLdsLimit = 160 * 1024;
constexpr int kChunkMin = 128;
constexpr int kChunkMax = 65536;

thread_local std::string g_error;

ba_status set_error(ba_status s, const std::string& m) {
  g_error = m;
  return s;
}

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Device copy of a std::vector inside one plan allocation.
struct Blob {
  std::vector<std::pair<size_t, std::vector<uint8_t>>> parts;
  size_t size = 0;
  template <typename T>
  size_t add(const std::vector<T>& v) {
    const size_t off = align_up(size);
    std::vector<uint8_t> bytes(v.size() * sizeof(T));
    if (!v.empty()) std::memcpy(bytes.data(), v.data(), bytes.size());
    parts.emplace_back(off, std::move(bytes));
    size = off + std::max<size_t>(parts.back().second.size(), 1);
    return off;
  }
};

struct DeviceTables {
  int tp = 0, chunk_obs = 0;
  int n_chunks = 0;
  int64_t part_elems = 0;
  void* mem = nullptr;
  WinDev* win = nullptr;
  int32_t* tile_lm_begin = nullptr;
  int32_t* chunk_window = nullptr;
  int32_t* chunk_tile_begin = nullptr;
  int64_t* chunk_part_off = nullptr;
  int32_t* chunk_order = nullptr;
  int32_t* pair_rec = nullptr;
  int32_t* tile_rec = nullptr;
  uint32_t* lists = nullptr;
  int32_t* win_order = nullptr;
  int cls_begin[kClasses + 1] = {0, 0, 0, 0, 0};
  int cls_win_begin[kClasses + 1] = {0, 0, 0, 0, 0};
  int cls_win_nf[kClasses] = {0, 0, 0, 0};
  int cls_nf[kClasses] = {0, 0, 0, 0};
  int list_bytes = 0;   // largest per-tile segment + product list
  int max_cpw = 0;      // largest chunk count of one window
  int cls_sum_slices[kClasses] = {0, 0, 0, 0};   // k_sum workgroups per window, per class
  int sum_slices = 0;
};

}  // namespace ba

using namespace ba;

struct ba_batch_s {
  std::vector<HostWindow> wins;
  int max_nf = 0, max_np = 0, max_nc = 0;
  int64_t n_poses = 0, n_points = 0, n_cams = 0, n_obs = 0, n_pairs = 0;
  int device = 0;
  void* mem = nullptr;   // plan arrays
  DevPlan plan{};
  DeviceTables tables[2];   // [0]: small tiles, [1]: large tiles
  // launch shape (ba_launch_config)
  int chunk_obs = 4096;
  int tile_pairs = 0;                      // 0: the largest tiles whose LDS fits
  int class_mult[kClasses] = {1, 1, 1, 1};  // work-item size per class, in chunk_obs
  int class_streams = 1;                   // size classes as concurrent chains
  // Set by the first launch made under stream capture: a graph may then hold
  // the launch tables' device pointers in its kernel arguments, so tables
  // replaced by ba_set_launch / ba_autotune are kept (in `retired`) until the
  // batch is destroyed instead of being freed.
  bool captured = false;
  std::vector<void*> retired;
  // the side streams of the size classes and their fork / join events (made
  // by the first launch of a plan with two or more size classes that is not
  // under stream capture)
  bool have_side = false;
  hipStream_t side[kSideStreams] = {};
  hipEvent_t ev_fork = nullptr, ev_join[kSideStreams] = {};
  std::mutex mu;
  ~ba_batch_s() {
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    for (int k = 0; k < kSideStreams; ++k) {
      if (ev_join[k]) (void)hipEventDestroy(ev_join[k]);
      if (side[k]) (void)hipStreamDestroy(side[k]);
    }
    if (mem) (void)hipFree(mem);
    for (auto& t : tables)
      if (t.mem) (void)hipFree(t.mem);
    for (void* m : retired) (void)hipFree(m);
  }
};

struct ba_window_s {
  HostWindow host;
  ba_batch_s* batch = nullptr;   // single-window batch, NULL when host-only
  ~ba_window_s() { delete batch; }
};

namespace {

ba_status hip_fail(hipError_t e, const char* what) {
  return set_error(BA_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

ba_status upload_tables(ba_batch_s* b, int which, int tp, int chunk_obs) {
  std::vector<const HostWindow*> ws;
  for (auto& w : b->wins) ws.push_back(&w);
  LaunchTables t;
  build_tiles(ws, tp, chunk_obs, t, b->class_mult);
  // per-window records with this table's chunk ranges
  std::vector<WinDev> wd(b->wins.size());
  int32_t po = 0, lo = 0, co = 0, oo = 0, pa = 0, so = 0;
  for (size_t i = 0; i < b->wins.size(); ++i) {
    const HostWindow& w = b->wins[i];
    WinDev& d = wd[i];
    d.n_poses = w.n_poses;
    d.n_points = w.n_points;
    d.n_cams = w.n_cams;
    d.n_free = w.n_free;
    d.pose_off = po;
    d.point_off = lo;
    d.cam_off = co;
    d.obs_off = oo;
    d.pair_off = pa;
    d.chunk_begin = t.win_chunk_begin[i];
    d.chunk_end = t.win_chunk_begin[i + 1];
    d.sum_off = so;
    d.sum_groups = sum_groups(d.chunk_end - d.chunk_begin);
    so += (int32_t)partial_elems(w.n_free);
    po += w.n_poses;
    lo += w.n_points;
    co += w.n_cams;
    oo += (int32_t)w.n_obs;
    pa += (int32_t)w.n_pairs();
  }
  Blob blob;
  const size_t o_win = blob.add(wd);
  const size_t o_tile = blob.add(t.tile_lm_begin);
  const size_t o_cw = blob.add(t.chunk_window);
  const size_t o_ct = blob.add(t.chunk_tile_begin);
  const size_t o_cp = blob.add(t.chunk_part_off);
  const size_t o_co = blob.add(t.chunk_order);
  const size_t o_wo = blob.add(t.win_order);
  const size_t o_pr = blob.add(t.pair_rec);
  const size_t o_tr = blob.add(t.tile_rec);
  const size_t o_ls = blob.add(t.lists);
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, blob.size);
  if (e != hipSuccess) return set_error(BA_ERR_OOM, "plan tables: hipMalloc failed");
  for (auto& p : blob.parts)
    if (!p.second.empty()) {
      e = hipMemcpy((char*)mem + p.first, p.second.data(), p.second.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        (void)hipFree(mem);
        return hip_fail(e, "plan tables upload");
      }
    }
  DeviceTables& D = b->tables[which];
  if (D.mem) {
    // hipFree waits for the device, so eager launches are done with the old
    // tables; a captured graph may still use them at any later replay
    if (b->captured) b->retired.push_back(D.mem);
    else (void)hipFree(D.mem);
  }
  D.mem = mem;
  D.tp = tp;
  D.chunk_obs = chunk_obs;
  D.n_chunks = t.n_chunks();
  D.part_elems = t.part_elems;
  D.win = (WinDev*)((char*)mem + o_win);
  D.tile_lm_begin = (int32_t*)((char*)mem + o_tile);
  D.chunk_window = (int32_t*)((char*)mem + o_cw);
  D.chunk_tile_begin = (int32_t*)((char*)mem + o_ct);
  D.chunk_part_off = (int64_t*)((char*)mem + o_cp);
  D.chunk_order = (int32_t*)((char*)mem + o_co);
  D.win_order = (int32_t*)((char*)mem + o_wo);
  D.pair_rec = (int32_t*)((char*)mem + o_pr);
  D.tile_rec = (int32_t*)((char*)mem + o_tr);
  D.lists = (uint32_t*)((char*)mem + o_ls);
  D.list_bytes = t.max_tile_words * 4 + 16;
  D.max_cpw = 0;
  for (size_t i = 0; i + 1 < t.win_chunk_begin.size(); ++i)
    D.max_cpw = std::max(D.max_cpw, t.win_chunk_begin[i + 1] - t.win_chunk_begin[i]);
  D.sum_slices = 1;
  for (int c = 0; c < kClasses; ++c) D.cls_sum_slices[c] = 1;
  for (size_t i = 0; i < b->wins.size(); ++i) {
    const int64_t ne = partial_elems(b->wins[i].n_free);
    const int per = sum_slice_entries(wd[i].sum_groups);
    const int n = (int)((ne + per - 1) / per);
    const int c = size_class(b->wins[i].n_free);
    D.cls_sum_slices[c] = std::max(D.cls_sum_slices[c], n);
    D.sum_slices = std::max(D.sum_slices, n);
  }
  for (int c = 0; c <= kClasses; ++c) D.cls_begin[c] = t.class_begin[c];
  for (int c = 0; c <= kClasses; ++c) D.cls_win_begin[c] = t.class_win_begin[c];
  for (int c = 0; c < kClasses; ++c) D.cls_win_nf[c] = t.class_win_nf[c];
  for (int c = 0; c < kClasses; ++c) D.cls_nf[c] = t.class_nf[c];
  return BA_OK;
}

// Work-item size of a new plan.  Many windows fill the GPU with whole windows,
// so their work items aim at n_obs / 1024 observations (1024 .. 8192).  A
// plan of one window has nothing to run beside it: its work items aim at one
// per CU (n_obs / 256, 128 .. 8192 observations; a work item is at least one
// tile), which spreads the window's latency-bound tiles over the chip.
int default_chunk_obs(int64_t n_obs, size_t n_windows) {
  if (n_windows == 1) return (int)std::min<int64_t>(8192, std::max<int64_t>(128, n_obs / 256));
  const int64_t c = n_obs / 1024;
  return (int)std::min<int64_t>(8192, std::max<int64_t>(1024, c));
}

ba_status batch_build(std::vector<HostWindow>&& wins, ba_batch_s** out) {
  std::unique_ptr<ba_batch_s> b(new ba_batch_s());
  b->wins = std::move(wins);
  std::vector<int32_t> free_slot, lm_pair_begin, pair_obs_begin, pair_lm, obs_perm;
  std::vector<uint8_t> lm_nfree, pair_pose, obs_cam;
  std::vector<double> cam;
  int32_t lm_base = 0, pair_base = 0, obs_base = 0;
  for (auto& w : b->wins) {
    b->max_nf = std::max(b->max_nf, w.n_free);
    b->max_np = std::max(b->max_np, w.n_poses);
    b->max_nc = std::max(b->max_nc, w.n_cams);
    for (int i = 0; i < w.n_poses; ++i) free_slot.push_back(w.free_slot[i]);
    cam.insert(cam.end(), w.cam.begin(), w.cam.end());
    for (int j = 0; j < w.n_points; ++j) {
      lm_pair_begin.push_back(pair_base + w.lm_pair_begin[j]);
      lm_nfree.push_back(w.lm_nfree[j]);
    }
    for (int64_t q = 0; q < w.n_pairs(); ++q) {
      pair_obs_begin.push_back(obs_base + w.pair_obs_begin[q]);
      pair_lm.push_back(lm_base + w.pair_lm[q]);
      pair_pose.push_back(w.pair_pose[q]);
    }
    obs_cam.insert(obs_cam.end(), w.obs_cam.begin(), w.obs_cam.end());
    obs_perm.insert(obs_perm.end(), w.perm.begin(), w.perm.end());
    lm_base += w.n_points;
    pair_base += (int32_t)w.n_pairs();
    obs_base += (int32_t)w.n_obs;
    b->n_poses += w.n_poses;
    b->n_points += w.n_points;
    b->n_cams += w.n_cams;
    b->n_obs += w.n_obs;
    b->n_pairs += w.n_pairs();
  }
  if (b->n_obs > (int64_t)INT32_MAX / 2 || b->n_pairs > (int64_t)INT32_MAX / 2)
    return set_error(BA_ERR_UNSUPPORTED, "batch too large for 32-bit indices");
  lm_pair_begin.push_back(pair_base);
  pair_obs_begin.push_back(obs_base);
  Blob blob;
  const size_t o_fs = blob.add(free_slot), o_cam = blob.add(cam), o_lpb = blob.add(lm_pair_begin),
               o_lnf = blob.add(lm_nfree), o_pob = blob.add(pair_obs_begin),
               o_plm = blob.add(pair_lm), o_pp = blob.add(pair_pose), o_oc = blob.add(obs_cam),
               o_op = blob.add(obs_perm);
  hipError_t e = hipGetDevice(&b->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipMalloc(&b->mem, blob.size);
  if (e != hipSuccess) return set_error(BA_ERR_OOM, "plan arrays: hipMalloc failed");
  for (auto& p : blob.parts)
    if (!p.second.empty()) {
      e = hipMemcpy((char*)b->mem + p.first, p.second.data(), p.second.size(), hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(e, "plan upload");
    }
  char* m = (char*)b->mem;
  b->plan.free_slot = (const int32_t*)(m + o_fs);
  b->plan.cam = (const double*)(m + o_cam);
  b->plan.lm_pair_begin = (const int32_t*)(m + o_lpb);
  b->plan.lm_nfree = (const uint8_t*)(m + o_lnf);
  b->plan.pair_obs_begin = (const int32_t*)(m + o_pob);
  b->plan.pair_lm = (const int32_t*)(m + o_plm);
  b->plan.pair_pose = (const uint8_t*)(m + o_pp);
  b->plan.obs_cam = (const uint8_t*)(m + o_oc);
  b->plan.obs_perm = (const int32_t*)(m + o_op);
  b->plan.n_windows = (int32_t)b->wins.size();
  b->chunk_obs = default_chunk_obs(b->n_obs, b->wins.size());
  ba_status s = upload_tables(b.get(), 0, kTileSmall, b->chunk_obs);
  if (s != BA_OK) return s;
  s = upload_tables(b.get(), 1, kTileLarge, b->chunk_obs);
  if (s != BA_OK) return s;
  *out = b.release();
  return BA_OK;
}

ba_status check_settings(const ba_settings* s) {
  if (!s) return set_error(BA_ERR_INVALID_ARG, "settings is NULL");
  if (s->max_iters < 0 || s->max_iters > 100000) return set_error(BA_ERR_INVALID_ARG, "max_iters out of range");
  if (s->precision != BA_FP64 && s->precision != BA_MIXED)
    return set_error(BA_ERR_INVALID_ARG, "unknown precision");
  if (!(s->lambda_init > 0) || !(s->lambda_up > 1) || !(s->lambda_down > 1) ||
      !(s->lambda_min > 0) || !(s->lambda_max >= s->lambda_min) || !std::isfinite(s->lambda_max))
    return set_error(BA_ERR_INVALID_ARG, "invalid lambda settings");
  if (!(s->grad_tol >= 0) || !std::isfinite(s->grad_tol) || !(s->step_tol >= 0) || !std::isfinite(s->step_tol))
    return set_error(BA_ERR_INVALID_ARG, "grad_tol and step_tol must be finite and >= 0");
  if (std::isnan(s->huber_delta) || !std::isfinite(s->min_depth))
    return set_error(BA_ERR_INVALID_ARG, "invalid huber_delta or min_depth");
  return BA_OK;
}

// Tile configuration for a precision: the large tiles when their LDS fits.
ba_status pick_config(const ba_batch_s* b, int precision, int* which) {
  const int nf = b->max_nf;
  if (precision == BA_FP64 && nf > kMaxFreeFp64)
    return set_error(BA_ERR_UNSUPPORTED, "BA_FP64 supports at most 29 free poses per window");
  auto fits = [&](int w) {
    const DeviceTables& t = b->tables[w];
    const size_t la = precision == BA_FP64
                          ? (t.tp == kTileLarge ? pass_a_lds<double, kTileLarge>(b->max_np, b->max_nc, nf, t.list_bytes, true)
                                                : pass_a_lds<double, kTileSmall>(b->max_np, b->max_nc, nf, t.list_bytes, true))
                          : (t.tp == kTileLarge ? pass_a_lds<float, kTileLarge>(b->max_np, b->max_nc, nf, t.list_bytes, true)
                                                : pass_a_lds<float, kTileSmall>(b->max_np, b->max_nc, nf, t.list_bytes, true));
    const size_t lb = precision == BA_FP64
                          ? (t.tp == kTileLarge ? pass_b_lds<double, kTileLarge>() : pass_b_lds<double, kTileSmall>())
                          : (t.tp == kTileLarge ? pass_b_lds<float, kTileLarge>() : pass_b_lds<float, kTileSmall>());
    return la <= kLdsLimit && lb <= kLdsLimit;
  };
  if (b->tile_pairs == kTileSmall) {
    if (!fits(0)) return set_error(BA_ERR_UNSUPPORTED, "window too large for LDS");
    *which = 0;
  } else if (b->tile_pairs == kTileLarge) {
    if (!fits(1)) return set_error(BA_ERR_UNSUPPORTED, "window too large for LDS with 256-pair tiles");
    *which = 1;
  } else if (fits(1)) {
    *which = 1;
  } else if (fits(0)) {
    *which = 0;
  } else {
    return set_error(BA_ERR_UNSUPPORTED, "window too large for LDS");
  }
  if (reduce_lds(nf) > kLdsLimit) return set_error(BA_ERR_UNSUPPORTED, "reduced system too large for LDS");
  return BA_OK;
}

struct Layout {
  size_t du, dv, w, poses_b, points_b, state, dp, ssum, part, cost_a, cost_b, flag_a, flag_b, gmax, smax, total;
};

Layout layout(const ba_batch_s* b, const DeviceTables& t, size_t real) {
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + std::max<size_t>(bytes, 1));
    return at;
  };
  L.du = take(real * b->n_obs);
  L.dv = take(real * b->n_obs);
  L.w = take(real * b->n_obs);
  L.poses_b = take(sizeof(double) * 12 * b->n_poses);
  L.points_b = take(sizeof(double) * 3 * b->n_points);
  L.state = take(sizeof(WinState) * b->wins.size());
  L.dp = take(sizeof(double) * kDpStride * b->wins.size());
  int64_t sum_elems = 0;
  for (auto& w : b->wins) sum_elems += partial_elems(w.n_free);
  L.ssum = take(sizeof(double) * sum_elems);
  L.part = take(real * t.part_elems);
  L.cost_a = take(sizeof(double) * t.n_chunks);
  L.cost_b = take(sizeof(double) * t.n_chunks);
  L.flag_a = take(sizeof(int32_t) * t.n_chunks);
  L.flag_b = take(sizeof(int32_t) * t.n_chunks);
  L.gmax = take(sizeof(double) * t.n_chunks);
  L.smax = take(sizeof(double) * t.n_chunks);
  L.total = o;
  return L;
}

template <typename Real>
DevWork<Real> make_work(const Layout& L, void* ws, bool has_w) {
  char* m = (char*)ws;
  DevWork<Real> K;
  K.du = (Real*)(m + L.du);
  K.dv = (Real*)(m + L.dv);
  K.w = has_w ? (Real*)(m + L.w) : nullptr;
  K.poses_b = (double*)(m + L.poses_b);
  K.points_b = (double*)(m + L.points_b);
  K.state = (WinState*)(m + L.state);
  K.dp = (double*)(m + L.dp);
  K.ssum = (double*)(m + L.ssum);
  K.part = (Real*)(m + L.part);
  K.part_cost_a = (double*)(m + L.cost_a);
  K.part_cost_b = (double*)(m + L.cost_b);
  K.part_flag_a = (int32_t*)(m + L.flag_a);
  K.part_flag_b = (int32_t*)(m + L.flag_b);
  K.part_gmax = (double*)(m + L.gmax);
  K.part_smax = (double*)(m + L.smax);
  K.vi_cost_a = nullptr;
  K.vi_cost_b = nullptr;
  K.vi_states = nullptr;
  K.vi_states_b = nullptr;
  return K;
}

ba_status ensure_attrs() {
  static std::once_flag once;
  static hipError_t err = hipSuccess;
  std::call_once(once, [] {
    hipError_t e;
    if ((e = set_attrs<double, kTileSmall, false>()) != hipSuccess) { err = e; return; }
    if ((e = set_attrs<double, kTileLarge, false>()) != hipSuccess) { err = e; return; }
    if ((e = set_attrs<float, kTileSmall, false>()) != hipSuccess) { err = e; return; }
    if ((e = set_attrs<float, kTileLarge, false>()) != hipSuccess) { err = e; return; }
    if ((e = set_attrs<double, kTileSmall, true>()) != hipSuccess) { err = e; return; }
    if ((e = set_attrs<double, kTileLarge, true>()) != hipSuccess) { err = e; return; }
    if ((e = set_attrs<float, kTileSmall, true>()) != hipSuccess) { err = e; return; }
    if ((e = set_attrs<float, kTileLarge, true>()) != hipSuccess) { err = e; return; }
  });
  if (err != hipSuccess) return hip_fail(err, "hipFuncSetAttribute");
  return BA_OK;
}

DevSettings dev_settings(const ba_settings* s) {
  DevSettings d;
  d.lambda_init = s->lambda_init;
  d.lambda_up = s->lambda_up;
  d.lambda_down = s->lambda_down;
  d.lambda_min = s->lambda_min;
  d.lambda_max = s->lambda_max;
  d.huber_delta = s->huber_delta;
  d.min_depth = s->min_depth;
  d.grad_tol = s->grad_tol;
  d.step_tol = s->step_tol;
  d.max_iters = s->max_iters;
  d.pad = 0;
  return d;
}

DevTiles dev_tiles(const DeviceTables& t) {
  DevTiles d;
  d.tile_lm_begin = t.tile_lm_begin;
  d.chunk_window = t.chunk_window;
  d.chunk_tile_begin = t.chunk_tile_begin;
  d.chunk_part_off = t.chunk_part_off;
  d.chunk_order = t.chunk_order;
  d.win_order = t.win_order;
  d.pair_rec = t.pair_rec;
  d.tile_rec = t.tile_rec;
  d.lists = t.lists;
  d.n_chunks = t.n_chunks;
  return d;
}

// The side streams of the size classes (default priority, no implicit
// synchronisation with other streams) and their events, made on the batch's
// device by the first launch that is not being captured; a capture before any
// such launch runs everything on the launch stream.  The caller holds b->mu.
ba_status ensure_side_stream(ba_batch_s* b, void* stream) {
  if (b->have_side) return BA_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  hipError_t e = hipStreamIsCapturing((hipStream_t)stream, &cs);
  if (e != hipSuccess) return hip_fail(e, "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone) return BA_OK;
  int cur = 0;
  if ((e = hipGetDevice(&cur)) != hipSuccess) return hip_fail(e, "hipGetDevice");
  if ((e = hipSetDevice(b->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
  for (int k = 0; k < kSideStreams && e == hipSuccess; ++k) {
    e = hipStreamCreateWithFlags(&b->side[k], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join[k], hipEventDisableTiming);
  }
  (void)hipSetDevice(cur);
  if (e != hipSuccess) {
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    b->ev_fork = nullptr;
    for (int k = 0; k < kSideStreams; ++k) {
      if (b->ev_join[k]) (void)hipEventDestroy(b->ev_join[k]);
      if (b->side[k]) (void)hipStreamDestroy(b->side[k]);
      b->ev_join[k] = nullptr;
      b->side[k] = nullptr;
    }
    return hip_fail(e, "side streams");
  }
  b->have_side = true;
  return BA_OK;
}

enum class Op { Solve, Adjoint, Timed };

// Inputs of a visual-inertial solve (ba_vi_solve).
struct ViInput {
  const double* preint;
  const double* gravity;   // host, 3
  double* states;          // device, 9 per pose
};

// Workspace bytes of the VI records after the window solve's own layout.
size_t vi_bytes(const ba_batch_s* b) {
  const HostWindow& w = b->wins[0];
  return align_up(sizeof(double) * (9 * (size_t)w.n_poses + 2 + vi_rec_doubles(w.n_poses, w.n_free)));
}

ba_status launch(ba_batch_s* b, const ba_settings* s, Op op, DevUser U, void* ws, size_t ws_bytes,
                 void* stream, bool has_w, double* stage_ms = nullptr, const ViInput* vin = nullptr) {
  int which = 0;
  ba_status st = pick_config(b, s->precision, &which);
  if (st != BA_OK) return st;
  const DeviceTables& t = b->tables[which];
  const size_t real = s->precision == BA_FP64 ? sizeof(double) : sizeof(float);
  const Layout L = layout(b, t, real);
  if (!ws) return set_error(BA_ERR_INVALID_ARG, "workspace is NULL");
  const size_t need = L.total + (vin ? vi_bytes(b) : 0);
  if (ws_bytes < need) return set_error(BA_ERR_WORKSPACE_TOO_SMALL, "workspace too small");
  if (((uintptr_t)ws) % 256 != 0) return set_error(BA_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if ((st = ensure_attrs()) != BA_OK) return st;
  LaunchArgs A;
  A.plan = b->plan;
  A.plan.win = t.win;
  A.tiles = dev_tiles(t);
  A.user = U;
  A.settings = dev_settings(s);
  A.max_nf = b->max_nf;
  for (int c = 0; c <= kClasses; ++c) A.cls_begin[c] = t.cls_begin[c];
  for (int c = 0; c <= kClasses; ++c) A.cls_win_begin[c] = t.cls_win_begin[c];
  for (int c = 0; c < kClasses; ++c) A.cls_win_nf[c] = t.cls_win_nf[c];
  for (int c = 0; c < kClasses; ++c) A.cls_nf[c] = t.cls_nf[c];
  A.dims.np = b->max_np;
  A.dims.nc = b->max_nc;
  A.list_bytes = t.list_bytes;
  A.max_cpw = t.max_cpw;
  for (int c = 0; c < kClasses; ++c) A.cls_sum_slices[c] = t.cls_sum_slices[c];
  A.sum_slices = t.sum_slices;
  A.stream = stream;
  int n_classes = 0;
  for (int c = 0; c < kClasses; ++c) n_classes += t.cls_win_begin[c + 1] > t.cls_win_begin[c];
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  unsigned long long cap_id = 0;
  hipError_t e = hipStreamGetCaptureInfo((hipStream_t)stream, &cs, &cap_id);
  if (e != hipSuccess) return hip_fail(e, "hipStreamGetCaptureInfo");
  if (cs != hipStreamCaptureStatusNone) b->captured = true;
  if (n_classes >= 2 && b->class_streams && (st = ensure_side_stream(b, stream)) != BA_OK) return st;
  // The side streams join a capture of `stream` through the fork event and
  // stay in it until that capture ends.  While they belong to another capture
  // (a call on another stream of this plan is being captured) the call runs
  // every class on `stream`, so that nothing is recorded into a foreign graph.
  bool use_side = b->have_side && b->class_streams;
  for (int k = 0; k < kSideStreams && use_side; ++k) {
    hipStreamCaptureStatus ss = hipStreamCaptureStatusNone;
    unsigned long long sid = 0;
    if ((e = hipStreamGetCaptureInfo(b->side[k], &ss, &sid)) != hipSuccess)
      return hip_fail(e, "hipStreamGetCaptureInfo");
    if (ss != hipStreamCaptureStatusNone && !(cs == hipStreamCaptureStatusActive && sid == cap_id))
      use_side = false;
  }
  A.side_stream = use_side ? (void*)b->side : nullptr;
  A.ev_fork = b->ev_fork;
  A.ev_join = (void*)b->ev_join;
  A.vi = nullptr;
  // visual-inertial: the VI records after the solve's own workspace
  ViArgs V{};
  double* vi_base = vin ? (double*)((char*)ws + L.total) : nullptr;
  if (vin) {
    const HostWindow& w0 = b->wins[0];
    V.win = t.win;
    V.win_order = t.win_order;
    V.free_slot = b->plan.free_slot;
    V.poses = U.poses;
    V.states = vin->states;
    V.states_b = vi_base;
    V.cost_a = vi_base + 9 * (size_t)w0.n_poses;
    V.cost_b = V.cost_a + 1;
    V.rec = V.cost_b + 1;
    V.preint = vin->preint;
    V.max_factors = w0.n_poses - 1;
    for (int k = 0; k < 3; ++k) V.g[k] = vin->gravity[k];
    A.vi = &V;
  }
  auto vi_work = [&](auto& K) {
    if (!vin) return;
    V.state = K.state;
    V.poses_b = K.poses_b;
    V.ssum = K.ssum;
    V.dp = K.dp;
    V.part_flag_a = K.part_flag_a;
    K.vi_cost_a = V.cost_a;
    K.vi_cost_b = V.cost_b;
    K.vi_states = V.states;
    K.vi_states_b = V.states_b;
  };
  if (s->precision == BA_FP64) {
    DevWork<double> K = make_work<double>(L, ws, has_w);
    vi_work(K);
    if (op == Op::Solve)
      e = t.tp == kTileLarge ? run_solve<double, kTileLarge>(A, K) : run_solve<double, kTileSmall>(A, K);
    else if (op == Op::Timed)
      e = t.tp == kTileLarge ? run_solve_timed<double, kTileLarge>(A, K, stage_ms)
                             : run_solve_timed<double, kTileSmall>(A, K, stage_ms);
    else
      e = t.tp == kTileLarge ? run_adjoint<double, kTileLarge>(A, K) : run_adjoint<double, kTileSmall>(A, K);
  } else {
    DevWork<float> K = make_work<float>(L, ws, has_w);
    vi_work(K);
    if (op == Op::Solve)
      e = t.tp == kTileLarge ? run_solve<float, kTileLarge>(A, K) : run_solve<float, kTileSmall>(A, K);
    else if (op == Op::Timed)
      e = t.tp == kTileLarge ? run_solve_timed<float, kTileLarge>(A, K, stage_ms)
                             : run_solve_timed<float, kTileSmall>(A, K, stage_ms);
    else
      e = t.tp == kTileLarge ? run_adjoint<float, kTileLarge>(A, K) : run_adjoint<float, kTileSmall>(A, K);
  }
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return BA_OK;
}

ba_batch_s* batch_of(ba_window w, ba_batch b) {
  if (w && !b) return w->batch;
  if (b && !w) return b;
  return nullptr;
}

// Address of `scratch` on one device, looked up once per device with that
// device current (each GPU holds its own copy at its own address).
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

ba_status scratch_on(int device, void** out) {
  if (device < 0 || device >= kMaxScratchDevices)
    return set_error(BA_ERR_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    const hipError_t e2 = hipSetDevice(cur);
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (e2 != hipSuccess) return hip_fail(e2, "hipSetDevice");
    if (!p) return set_error(BA_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return BA_OK;
}

}  // namespace

extern "C" {

const char* ba_status_string(ba_status s) {
  switch (s) {
    case BA_OK: return "ok";
    case BA_ERR_INVALID_ARG: return "invalid argument";
    case BA_ERR_OOM: return "out of memory";
    case BA_ERR_HIP: return "HIP runtime error";
    case BA_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
    case BA_ERR_UNSUPPORTED: return "unsupported structure";
    case BA_ERR_STATE: return "handle not usable for this call";
  }
  return "unknown status";
}

const char* ba_last_error(void) { return g_error.c_str(); }

// ---------------------------------------------------------------------------
// motion-only solves
// ---------------------------------------------------------------------------

struct ba_rig_s {
  int n_cams = 0;
  int device = 0;
  double* cams = nullptr;   // device, n_cams * 16
  int waves_per_frame = 0;  // 0: chosen per launch
  ~ba_rig_s() {
    if (cams) (void)hipFree(cams);
  }
};

ba_status ba_rig_create(int32_t n_cams, const double* intrinsics, const double* extrinsics,
                        ba_rig* out) {
  if (!out) return set_error(BA_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (n_cams < 1 || !intrinsics) return set_error(BA_ERR_INVALID_ARG, "n_cams < 1 or intrinsics is NULL");
  if (n_cams > kMaxCams) return set_error(BA_ERR_UNSUPPORTED, "more than 32 cameras in a rig");
  std::vector<double> cam;
  const std::string m = pack_cameras(n_cams, intrinsics, extrinsics, cam);
  if (!m.empty()) return set_error(BA_ERR_INVALID_ARG, m);
  std::unique_ptr<ba_rig_s> r(new ba_rig_s);
  r->n_cams = n_cams;
  hipError_t e = hipGetDevice(&r->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipMalloc(&r->cams, cam.size() * sizeof(double));
  if (e != hipSuccess) {
    r->cams = nullptr;
    return set_error(BA_ERR_OOM, "rig: hipMalloc failed");
  }
  e = hipMemcpy(r->cams, cam.data(), cam.size() * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "rig upload");
  *out = r.release();
  return BA_OK;
}

void ba_rig_destroy(ba_rig rig) { delete rig; }

ba_status ba_rig_set_waves_per_frame(ba_rig rig, int32_t waves_per_frame) {
  if (!rig) return set_error(BA_ERR_INVALID_ARG, "rig is NULL");
  if (waves_per_frame != 0 && waves_per_frame != 1 && waves_per_frame != 2 && waves_per_frame != 4)
    return set_error(BA_ERR_INVALID_ARG, "waves per frame must be 0, 1, 2 or 4");
  rig->waves_per_frame = waves_per_frame;
  return BA_OK;
}

ba_status ba_pnp_solve(ba_rig rig, const ba_settings* s, int32_t n_frames, int64_t n_obs,
                       int64_t n_points, const int32_t* frame_obs_begin, double* poses,
                       const double* points, const int32_t* obs_point, const int32_t* obs_cam,
                       const double* obs_uv, const double* obs_w, const double* frame_transform,
                       ba_report* reports, ba_iter_trace* traces, void* stream) {
  if (!rig) return set_error(BA_ERR_INVALID_ARG, "rig is NULL");
  ba_status st = check_settings(s);
  if (st != BA_OK) return st;
  if (n_frames < 0 || n_obs < 0 || n_points < 0) return set_error(BA_ERR_INVALID_ARG, "negative size");
  if (n_obs > (int64_t)INT32_MAX) return set_error(BA_ERR_UNSUPPORTED, "too many observations");
  if (n_frames == 0) return BA_OK;
  if (!frame_obs_begin || !poses || (n_points > 0 && !points) ||
      (n_obs > 0 && (!obs_point || !obs_uv)))
    return set_error(BA_ERR_INVALID_ARG, "NULL device array");
  hipError_t e = hipSetDevice(rig->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  PnpArgs A;
  A.cams = rig->cams;
  A.n_cams = rig->n_cams;
  A.n_frames = n_frames;
  A.n_obs = n_obs;
  A.n_points = n_points;
  A.frame_obs_begin = frame_obs_begin;
  A.poses = poses;
  A.points = points;
  A.obs_point = obs_point;
  A.obs_cam = obs_cam;
  A.obs_uv = obs_uv;
  A.obs_w = obs_w;
  A.frame_transform = frame_transform;
  A.reports = reports;
  A.traces = traces;
  A.settings = dev_settings(s);
  A.waves_per_frame = rig->waves_per_frame ? rig->waves_per_frame : pnp_waves_per_frame(n_frames, n_obs);
  A.stream = stream;
  e = s->precision == BA_FP64 ? run_pnp<double>(A) : run_pnp<float>(A);
  if (e != hipSuccess) return hip_fail(e, "motion-only launch");
  return BA_OK;
}

ba_status ba_triangulate(ba_rig rig, const ba_settings* s, int32_t n_points, int64_t n_obs,
                         int32_t n_poses, const int32_t* point_obs_begin, const double* poses,
                         const int32_t* obs_pose, const int32_t* obs_cam, const double* obs_uv,
                         const double* obs_w, double* points, ba_report* reports,
                         ba_iter_trace* traces, void* stream) {
  if (!rig) return set_error(BA_ERR_INVALID_ARG, "rig is NULL");
  ba_status st = check_settings(s);
  if (st != BA_OK) return st;
  if (n_points < 0 || n_obs < 0 || n_poses < 0) return set_error(BA_ERR_INVALID_ARG, "negative size");
  if (n_obs > (int64_t)INT32_MAX) return set_error(BA_ERR_UNSUPPORTED, "too many observations");
  if (n_points == 0) return BA_OK;
  if (!point_obs_begin || !points || (n_poses > 0 && !poses) || (n_obs > 0 && (!obs_pose || !obs_uv)))
    return set_error(BA_ERR_INVALID_ARG, "NULL device array");
  hipError_t e = hipSetDevice(rig->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  TriArgs A;
  A.cams = rig->cams;
  A.n_cams = rig->n_cams;
  A.n_points = n_points;
  A.n_poses = n_poses;
  A.n_obs = n_obs;
  A.point_obs_begin = point_obs_begin;
  A.poses = poses;
  A.obs_pose = obs_pose;
  A.obs_cam = obs_cam;
  A.obs_uv = obs_uv;
  A.obs_w = obs_w;
  A.points = points;
  A.reports = reports;
  A.traces = traces;
  A.settings = dev_settings(s);
  A.stream = stream;
  e = s->precision == BA_FP64 ? run_triangulate<double>(A) : run_triangulate<float>(A);
  if (e != hipSuccess) return hip_fail(e, "triangulation launch");
  return BA_OK;
}

// ---------------------------------------------------------------------------
// pose-graph optimisation
// ---------------------------------------------------------------------------

struct ba_graph_s {
  PgoPlan plan;
  int device = 0;
  void* mem = nullptr;
  PgoDev dev{};
  ~ba_graph_s() {
    if (mem) (void)hipFree(mem);
  }
};

ba_status ba_graph_create(int32_t n_poses, int32_t n_edges, const int32_t* edge_i,
                          const int32_t* edge_j, const uint8_t* pose_fixed, int32_t flags,
                          ba_graph* out) {
  if (!out) return set_error(BA_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (flags & ~BA_CREATE_HOST_ONLY) return set_error(BA_ERR_INVALID_ARG, "unknown flags");
  std::unique_ptr<ba_graph_s> g(new (std::nothrow) ba_graph_s());
  if (!g) return set_error(BA_ERR_OOM, "host allocation failed");
  const std::string err = build_pgo_plan(n_poses, n_edges, edge_i, edge_j, pose_fixed, g->plan);
  if (!err.empty()) return set_error(BA_ERR_INVALID_ARG, err);
  const PgoPlan& P = g->plan;
  if (flags & BA_CREATE_HOST_ONLY) {
    *out = g.release();
    return BA_OK;
  }
  Blob blob;
  const size_t o_cop = blob.add(P.col_of_pose), o_poc = blob.add(P.pose_of_col),
               o_lev = blob.add(P.lev_ptr), o_bp = blob.add(P.blk_ptr), o_br = blob.add(P.blk_row),
               o_up = blob.add(P.upd_ptr), o_ua = blob.add(P.upd_a), o_ub = blob.add(P.upd_b),
               o_fp = blob.add(P.fwd_ptr), o_fb = blob.add(P.fwd_blk), o_fc = blob.add(P.fwd_col),
               o_ap = blob.add(P.asm_ptr), o_ae = blob.add(P.asm_edge), o_rp = blob.add(P.rhs_ptr),
               o_re = blob.add(P.rhs_edge), o_ei = blob.add(P.edge_i), o_ej = blob.add(P.edge_j),
               o_bc = blob.add(P.blk_col), o_cp = blob.add(P.chunk_ptr), o_cb = blob.add(P.chunk_blk),
               o_fcp = blob.add(P.fchunk_ptr), o_fcc = blob.add(P.fchunk_col),
               o_cab = blob.add(P.chunk_ab), o_fbc = blob.add(P.fchunk_bc);
  hipError_t e = hipGetDevice(&g->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  e = hipMalloc(&g->mem, blob.size);
  if (e != hipSuccess) {
    g->mem = nullptr;
    return set_error(BA_ERR_OOM, "graph plan: hipMalloc failed");
  }
  for (auto& part : blob.parts)
    if (!part.second.empty()) {
      e = hipMemcpy((char*)g->mem + part.first, part.second.data(), part.second.size(),
                    hipMemcpyHostToDevice);
      if (e != hipSuccess) return hip_fail(e, "graph plan upload");
    }
  auto at = [&](size_t off) { return (const int32_t*)((char*)g->mem + off); };
  PgoDev& D = g->dev;
  D.n_poses = P.n_poses;
  D.n_edges = P.n_edges;
  D.n_free = P.n_free;
  D.n_levels = P.n_levels;
  D.n_blocks = P.n_blocks();
  D.col_of_pose = at(o_cop);
  D.pose_of_col = at(o_poc);
  D.lev_ptr = at(o_lev);
  D.blk_ptr = at(o_bp);
  D.blk_row = at(o_br);
  D.upd_ptr = at(o_up);
  D.upd_a = at(o_ua);
  D.upd_b = at(o_ub);
  D.fwd_ptr = at(o_fp);
  D.fwd_blk = at(o_fb);
  D.fwd_col = at(o_fc);
  D.asm_ptr = at(o_ap);
  D.asm_edge = at(o_ae);
  D.rhs_ptr = at(o_rp);
  D.rhs_edge = at(o_re);
  D.edge_i = at(o_ei);
  D.edge_j = at(o_ej);
  D.blk_col = at(o_bc);
  D.chunk_ptr = at(o_cp);
  D.chunk_blk = at(o_cb);
  D.fchunk_ptr = at(o_fcp);
  D.fchunk_col = at(o_fcc);
  D.chunk_ab = at(o_cab);
  D.fchunk_bc = at(o_fbc);
  D.n_chunks = (int)P.chunk_blk.size();
  D.n_fchunks = (int)P.fchunk_col.size();
  D.n_wide = P.n_wide;
  *out = g.release();
  return BA_OK;
}

void ba_graph_destroy(ba_graph g) { delete g; }

ba_status ba_graph_info(ba_graph g, int32_t* n_free, int32_t* n_levels, int32_t* n_blocks) {
  if (!g) return set_error(BA_ERR_INVALID_ARG, "graph is NULL");
  if (n_free) *n_free = g->plan.n_free;
  if (n_levels) *n_levels = g->plan.n_levels;
  if (n_blocks) *n_blocks = g->plan.n_blocks();
  return BA_OK;
}

ba_status ba_graph_plan_array(ba_graph g, int32_t which, const int32_t** data, int64_t* len) {
  if (!g || !data || !len) return set_error(BA_ERR_INVALID_ARG, "NULL argument");
  const PgoPlan& P = g->plan;
  const std::vector<int32_t>* v[] = {&P.col_of_pose, &P.pose_of_col, &P.lev_ptr, &P.blk_ptr,
                                     &P.blk_row, &P.upd_ptr, &P.upd_a, &P.upd_b, &P.fwd_ptr,
                                     &P.fwd_blk, &P.fwd_col, &P.asm_ptr, &P.asm_edge, &P.rhs_ptr,
                                     &P.rhs_edge};
  if (which < 0 || which >= (int)(sizeof(v) / sizeof(v[0])))
    return set_error(BA_ERR_INVALID_ARG, "unknown plan table");
  *data = v[which]->data();
  *len = (int64_t)v[which]->size();
  return BA_OK;
}

ba_status ba_graph_workspace_size(ba_graph g, size_t* bytes) {
  if (!g || !bytes) return set_error(BA_ERR_INVALID_ARG, "NULL argument");
  *bytes = pgo_workspace_bytes(g->plan);
  return BA_OK;
}

ba_status ba_pgo_solve(ba_graph g, const ba_settings* s, double* poses, const double* deltas,
                       const double* edge_w, void* workspace, size_t ws_bytes, ba_report* report,
                       ba_iter_trace* traces, void* stream) {
  if (!g) return set_error(BA_ERR_INVALID_ARG, "graph is NULL");
  if (!g->mem) return set_error(BA_ERR_STATE, "graph planned host-only");
  ba_status st = check_settings(s);
  if (st != BA_OK) return st;
  if (!poses || (g->plan.n_edges > 0 && !deltas)) return set_error(BA_ERR_INVALID_ARG, "NULL device array");
  const size_t need = pgo_workspace_bytes(g->plan);
  if (!workspace || ws_bytes < need)
    return set_error(BA_ERR_WORKSPACE_TOO_SMALL, "workspace below ba_graph_workspace_size");
  if (((uintptr_t)workspace) & 255) return set_error(BA_ERR_INVALID_ARG, "workspace not 256-byte aligned");
  hipError_t e = hipSetDevice(g->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  PgoArgs A;
  A.G = g->dev;
  A.W = pgo_carve(g->plan, workspace);
  A.poses = poses;
  A.deltas = deltas;
  A.edge_w = edge_w;
  A.report = report;
  A.traces = traces;
  A.settings = dev_settings(s);
  A.stream = stream;
  A.wide_tasks = g->plan.wide_tasks.data();
  e = run_pgo(A);
  if (e != hipSuccess) return hip_fail(e, "pose-graph launch");
  return BA_OK;
}

ba_status ba_window_create(int32_t n_poses, int32_t n_points, int32_t n_cams, int64_t n_obs,
                           const int32_t* obs_pose, const int32_t* obs_point,
                           const int32_t* obs_cam, const uint8_t* pose_fixed,
                           const double* intrinsics, const double* extrinsics, int32_t flags,
                           ba_window* out) {
  if (!out) return set_error(BA_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (flags & ~BA_CREATE_HOST_ONLY) return set_error(BA_ERR_INVALID_ARG, "unknown flags");
  std::unique_ptr<ba_window_s> w(new (std::nothrow) ba_window_s());
  if (!w) return set_error(BA_ERR_OOM, "host allocation failed");
  int code = 0;
  const std::string err = build_window(n_poses, n_points, n_cams, n_obs, obs_pose, obs_point,
                                       obs_cam, pose_fixed, intrinsics, extrinsics, w->host, &code);
  if (code != 0) return set_error((ba_status)code, err);
  if (!(flags & BA_CREATE_HOST_ONLY)) {
    std::vector<HostWindow> one(1, w->host);
    ba_status s = batch_build(std::move(one), &w->batch);
    if (s != BA_OK) return s;
  }
  *out = w.release();
  return BA_OK;
}

void ba_window_destroy(ba_window w) { delete w; }

static void fill_info(const HostWindow& h, int n_tiles, int n_chunks, ba_plan_info* info) {
  info->n_poses = h.n_poses;
  info->n_points = h.n_points;
  info->n_cams = h.n_cams;
  info->n_free = h.n_free;
  info->n_obs = h.n_obs;
  info->n_pairs = h.n_pairs();
  info->n_tiles = n_tiles;
  info->n_chunks = n_chunks;
  info->schur_blocks = h.schur_blocks;
  info->n_free_pairs = h.n_free_pairs;
}

ba_status ba_window_info(ba_window w, ba_plan_info* info) {
  if (!w || !info) return set_error(BA_ERR_INVALID_ARG, "NULL argument");
  std::vector<const HostWindow*> one{&w->host};
  LaunchTables t;
  build_tiles(one, kTileLarge, default_chunk_obs(w->host.n_obs, 1), t);
  fill_info(w->host, t.n_tiles(), t.n_chunks(), info);
  return BA_OK;
}

ba_status ba_window_order(ba_window w, int64_t* perm) {
  if (!w || (!perm && w->host.n_obs > 0)) return set_error(BA_ERR_INVALID_ARG, "NULL argument");
  for (int64_t k = 0; k < w->host.n_obs; ++k) perm[k] = w->host.perm[k];
  return BA_OK;
}

ba_status ba_batch_create(int32_t n_windows, const ba_window* windows, ba_batch* out) {
  if (!out || !windows || n_windows < 1) return set_error(BA_ERR_INVALID_ARG, "invalid arguments");
  *out = nullptr;
  std::vector<HostWindow> ws;
  ws.reserve(n_windows);
  for (int i = 0; i < n_windows; ++i) {
    if (!windows[i]) return set_error(BA_ERR_INVALID_ARG, "NULL window in list");
    ws.push_back(windows[i]->host);
  }
  ba_batch_s* b = nullptr;
  ba_status s = batch_build(std::move(ws), &b);
  if (s != BA_OK) return s;
  *out = b;
  return BA_OK;
}

void ba_batch_destroy(ba_batch b) { delete b; }

ba_status ba_batch_info(ba_batch b, int32_t window, ba_plan_info* info) {
  if (!b || !info || window < 0 || window >= (int32_t)b->wins.size())
    return set_error(BA_ERR_INVALID_ARG, "invalid arguments");
  const DeviceTables& t = b->tables[1];
  fill_info(b->wins[window], 0, t.n_chunks, info);
  return BA_OK;
}

ba_status ba_workspace_size(ba_window w, ba_batch b, const ba_settings* s, size_t* bytes) {
  if (!bytes) return set_error(BA_ERR_INVALID_ARG, "bytes is NULL");
  if (w && !w->batch && !b) return set_error(BA_ERR_STATE, "host-only window");
  ba_batch_s* bb = batch_of(w, b);
  if (!bb) return set_error(BA_ERR_INVALID_ARG, "exactly one of w, b must be given");
  ba_status st = check_settings(s);
  if (st != BA_OK) return st;
  int which = 0;
  if ((st = pick_config(bb, s->precision, &which)) != BA_OK) return st;
  const size_t real = s->precision == BA_FP64 ? sizeof(double) : sizeof(float);
  *bytes = layout(bb, bb->tables[which], real).total;
  return BA_OK;
}

ba_status ba_solve_batched(ba_batch b, const ba_settings* s, double* poses, double* points,
                           const double* obs_uv, const double* obs_w, void* workspace,
                           size_t ws_bytes, ba_report* reports, ba_iter_trace* traces,
                           void* stream) {
  if (!b) return set_error(BA_ERR_INVALID_ARG, "batch is NULL");
  ba_status st = check_settings(s);
  if (st != BA_OK) return st;
  if (!poses || (!points && b->n_points > 0) || (!obs_uv && b->n_obs > 0) || !reports)
    return set_error(BA_ERR_INVALID_ARG, "NULL device array");
  DevUser U{};
  U.poses = poses;
  U.points = points;
  U.obs_uv = obs_uv;
  U.obs_w = obs_w;
  U.reports = reports;
  U.traces = traces;
  std::lock_guard<std::mutex> lk(b->mu);
  return launch(b, s, Op::Solve, U, workspace, ws_bytes, stream, obs_w != nullptr);
}

ba_status ba_solve(ba_window w, const ba_settings* s, double* poses, double* points,
                   const double* obs_uv, const double* obs_w, void* workspace, size_t ws_bytes,
                   ba_report* report, ba_iter_trace* trace, void* stream) {
  if (!w) return set_error(BA_ERR_INVALID_ARG, "window is NULL");
  if (!w->batch) return set_error(BA_ERR_STATE, "host-only window cannot be solved");
  return ba_solve_batched(w->batch, s, poses, points, obs_uv, obs_w, workspace, ws_bytes, report,
                          trace, stream);
}

ba_status ba_solve_noalloc(ba_window w, const ba_settings* s, double* poses, double* points,
                           const double* obs_uv, const double* obs_w, ba_report* report,
                           ba_iter_trace* trace, void* stream) {
  if (!w) return set_error(BA_ERR_INVALID_ARG, "window is NULL");
  if (!w->batch) return set_error(BA_ERR_STATE, "host-only window cannot be solved");
  size_t need = 0;
  ba_status st = ba_workspace_size(w, nullptr, s, &need);
  if (st != BA_OK) return st;
  if (need > (size_t)BA_NOALLOC_SCRATCH_BYTES)
    return set_error(BA_ERR_WORKSPACE_TOO_SMALL,
                     "window needs " + std::to_string(need) + " bytes of workspace; ba_solve_noalloc " +
                         "holds at most " + std::to_string((size_t)BA_NOALLOC_SCRATCH_BYTES) +
                         " per device (use ba_solve with a workspace)");
  void* ptr = nullptr;
  if ((st = scratch_on(w->batch->device, &ptr)) != BA_OK) return st;
  return ba_solve_batched(w->batch, s, poses, points, obs_uv, obs_w, ptr,
                          (size_t)BA_NOALLOC_SCRATCH_BYTES, report, trace, stream);
}

ba_status ba_vi_preintegrate(int32_t n_factors, const int32_t* sample_begin, const double* gyro,
                             const double* accel, double dt, const double* bias_bar, const double* noise,
                             double* preint, void* stream) {
  if (n_factors < 0) return set_error(BA_ERR_INVALID_ARG, "negative factor count");
  if (n_factors == 0) return BA_OK;
  if (!sample_begin || !gyro || !accel || !bias_bar || !noise || !preint)
    return set_error(BA_ERR_INVALID_ARG, "NULL argument");
  if (!(dt > 0) || !std::isfinite(dt)) return set_error(BA_ERR_INVALID_ARG, "dt must be positive");
  for (int k = 0; k < 4; ++k)
    if (!(noise[k] > 0) || !std::isfinite(noise[k]))
      return set_error(BA_ERR_INVALID_ARG, "noise densities must be positive");
  const hipError_t e = launch_vi_preint(n_factors, sample_begin, gyro, accel, dt, bias_bar, noise, preint,
                                        (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "preintegration launch");
  return BA_OK;
}

ba_status ba_vi_workspace_size(ba_window w, const ba_settings* s, size_t* bytes) {
  if (!bytes) return set_error(BA_ERR_INVALID_ARG, "bytes is NULL");
  if (!w) return set_error(BA_ERR_INVALID_ARG, "window is NULL");
  if (!w->batch) return set_error(BA_ERR_STATE, "host-only window");
  const HostWindow& h = w->batch->wins[0];
  if (h.n_poses < 2 || h.n_poses > kViMaxStates)
    return set_error(BA_ERR_UNSUPPORTED, "visual-inertial windows hold 2 to 24 keyframes");
  size_t base = 0;
  ba_status st = ba_workspace_size(w, nullptr, s, &base);
  if (st != BA_OK) return st;
  *bytes = base + vi_bytes(w->batch);
  return BA_OK;
}

ba_status ba_vi_solve(ba_window w, const ba_settings* s, const double* preint, const double* gravity,
                      double* poses, double* points, double* states, const double* obs_uv, const double* obs_w,
                      void* workspace, size_t ws_bytes, ba_report* report, ba_iter_trace* trace, void* stream) {
  if (!w) return set_error(BA_ERR_INVALID_ARG, "window is NULL");
  if (!w->batch) return set_error(BA_ERR_STATE, "host-only window cannot be solved");
  ba_status st = check_settings(s);
  if (st != BA_OK) return st;
  ba_batch_s* b = w->batch;
  const HostWindow& h = b->wins[0];
  if (h.n_poses < 2 || h.n_poses > kViMaxStates)
    return set_error(BA_ERR_UNSUPPORTED, "visual-inertial windows hold 2 to 24 keyframes");
  if (s->grad_tol != 0 || s->step_tol != 0)
    return set_error(BA_ERR_UNSUPPORTED, "visual-inertial solves run a fixed number of attempts (tolerances 0)");
  if (!preint || !gravity || !states || !poses || (!points && b->n_points > 0) || (!obs_uv && b->n_obs > 0) ||
      !report)
    return set_error(BA_ERR_INVALID_ARG, "NULL argument");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(gravity[k])) return set_error(BA_ERR_INVALID_ARG, "non-finite gravity");
  DevUser U{};
  U.poses = poses;
  U.points = points;
  U.obs_uv = obs_uv;
  U.obs_w = obs_w;
  U.reports = report;
  U.traces = trace;
  ViInput vin{preint, gravity, states};
  std::lock_guard<std::mutex> lk(b->mu);
  return launch(b, s, Op::Solve, U, workspace, ws_bytes, stream, obs_w != nullptr, nullptr, &vin);
}

ba_status ba_adjoint(ba_window w, ba_batch b, const ba_settings* s, const double* poses,
                     const double* points, const double* obs_uv, const double* obs_w,
                     const double* grad_poses, const double* grad_points, double* grad_uv,
                     double* grad_w, void* workspace, size_t ws_bytes, ba_report* reports,
                     void* stream) {
  if (w && !w->batch && !b) return set_error(BA_ERR_STATE, "host-only window");
  ba_batch_s* bb = batch_of(w, b);
  if (!bb) return set_error(BA_ERR_INVALID_ARG, "exactly one of w, b must be given");
  ba_status st = check_settings(s);
  if (st != BA_OK) return st;
  if (!poses || (!points && bb->n_points > 0) || (!obs_uv && bb->n_obs > 0) || !grad_poses ||
      (!grad_uv && bb->n_obs > 0))
    return set_error(BA_ERR_INVALID_ARG, "NULL device array");
  DevUser U{};
  U.poses = const_cast<double*>(poses);
  U.points = const_cast<double*>(points);
  U.obs_uv = obs_uv;
  U.obs_w = obs_w;
  U.reports = reports;
  U.grad_poses = grad_poses;
  U.grad_points = grad_points;
  U.grad_uv = grad_uv;
  U.grad_w = grad_w;
  std::lock_guard<std::mutex> lk(bb->mu);
  return launch(bb, s, Op::Adjoint, U, workspace, ws_bytes, stream, obs_w != nullptr);
}

ba_status ba_profile_stages(ba_batch b, const ba_settings* s, double* poses, double* points,
                            const double* obs_uv, const double* obs_w, void* workspace,
                            size_t ws_bytes, ba_report* reports, void* stream, double* stage_ms) {
  if (!b || !stage_ms) return set_error(BA_ERR_INVALID_ARG, "NULL argument");
  ba_status st = check_settings(s);
  if (st != BA_OK) return st;
  if (!poses || (!points && b->n_points > 0) || (!obs_uv && b->n_obs > 0) || !reports)
    return set_error(BA_ERR_INVALID_ARG, "NULL device array");
  DevUser U{};
  U.poses = poses;
  U.points = points;
  U.obs_uv = obs_uv;
  U.obs_w = obs_w;
  U.reports = reports;
  std::lock_guard<std::mutex> lk(b->mu);
  return launch(b, s, Op::Timed, U, workspace, ws_bytes, stream, obs_w != nullptr, stage_ms);
}

ba_status ba_set_launch(ba_batch b, int32_t chunk_obs) {
  if (!b) return set_error(BA_ERR_INVALID_ARG, "batch is NULL");
  ba_launch_config c;
  ba_status s = ba_get_launch(b, &c);
  if (s != BA_OK) return s;
  c.chunk_obs = chunk_obs;
  return ba_set_launch_config(b, &c);
}

ba_status ba_get_launch(ba_batch b, ba_launch_config* cfg) {
  if (!b || !cfg) return set_error(BA_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(b->mu);
  cfg->chunk_obs = b->chunk_obs;
  cfg->tile_pairs = b->tile_pairs;
  for (int c = 0; c < kClasses; ++c) cfg->class_chunk_mult[c] = b->class_mult[c];
  cfg->class_streams = b->class_streams;
  return BA_OK;
}

ba_status ba_set_launch_config(ba_batch b, const ba_launch_config* cfg) {
  if (!b || !cfg) return set_error(BA_ERR_INVALID_ARG, "NULL argument");
  if (cfg->chunk_obs < kChunkMin || cfg->chunk_obs > kChunkMax)
    return set_error(BA_ERR_INVALID_ARG, "chunk_obs out of range");
  if (cfg->tile_pairs != 0 && cfg->tile_pairs != kTileSmall && cfg->tile_pairs != kTileLarge)
    return set_error(BA_ERR_INVALID_ARG, "tile_pairs must be 0, 64 or 256");
  for (int c = 0; c < kClasses; ++c)
    if (cfg->class_chunk_mult[c] < 1 || cfg->class_chunk_mult[c] > 4)
      return set_error(BA_ERR_INVALID_ARG, "class_chunk_mult out of range (1..4)");
  if (cfg->class_streams != 0 && cfg->class_streams != 1)
    return set_error(BA_ERR_INVALID_ARG, "class_streams must be 0 or 1");
  std::lock_guard<std::mutex> lk(b->mu);
  const int old_mult[kClasses] = {b->class_mult[0], b->class_mult[1], b->class_mult[2], b->class_mult[3]};
  const int old_tp = b->tile_pairs;
  for (int c = 0; c < kClasses; ++c) b->class_mult[c] = cfg->class_chunk_mult[c];
  b->tile_pairs = cfg->tile_pairs;
  ba_status s = upload_tables(b, 0, kTileSmall, cfg->chunk_obs);
  if (s == BA_OK) s = upload_tables(b, 1, kTileLarge, cfg->chunk_obs);
  if (s != BA_OK) {   // put the previous shape back (best effort: this only fails on OOM)
    for (int c = 0; c < kClasses; ++c) b->class_mult[c] = old_mult[c];
    b->tile_pairs = old_tp;
    (void)upload_tables(b, 0, kTileSmall, b->chunk_obs);
    (void)upload_tables(b, 1, kTileLarge, b->chunk_obs);
    return s;
  }
  b->chunk_obs = cfg->chunk_obs;
  b->class_streams = cfg->class_streams;
  return BA_OK;
}

ba_status ba_autotune(ba_batch b, const ba_settings* s, double* poses, double* points,
                      const double* obs_uv, const double* obs_w, void* workspace, size_t ws_bytes,
                      void* stream, int32_t* chosen_chunk_obs) {
  if (!b) return set_error(BA_ERR_INVALID_ARG, "batch is NULL");
  ba_status st = check_settings(s);
  if (st != BA_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  // cache key: device, precision, window count, size bucket, largest window
  // and the class mix (windows and observation bucket of each size class)
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, b->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
  auto bucket_of = [](int64_t n) {
    int k = 0;
    for (; n > 1; n >>= 1) ++k;
    return k;
  };
  int64_t cls_win[kClasses] = {0, 0, 0, 0}, cls_obs[kClasses] = {0, 0, 0, 0};
  for (const HostWindow& w : b->wins) {
    ++cls_win[size_class(w.n_free)];
    cls_obs[size_class(w.n_free)] += w.n_obs;
  }
  std::ostringstream keyss;
  keyss << prop.gcnArchName << "|" << s->precision << "|" << b->wins.size() << "|" << bucket_of(b->n_obs) << "|"
        << b->max_nf;
  for (int c = 0; c < kClasses; ++c) keyss << "|" << cls_win[c] << ":" << bucket_of(cls_obs[c]);
  const std::string key = keyss.str();
  const char* cache = std::getenv("BA_TUNE_CACHE");
  if (cache) {
    std::ifstream in(cache);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      ba_launch_config c{};
      if (!(ls >> k >> c.chunk_obs >> c.tile_pairs >> c.class_chunk_mult[0] >> c.class_chunk_mult[1] >>
            c.class_chunk_mult[2] >> c.class_chunk_mult[3] >> c.class_streams))
        continue;
      if (k != key) continue;
      if (ba_set_launch_config(b, &c) == BA_OK) {
        if (chosen_chunk_obs) *chosen_chunk_obs = c.chunk_obs;
        return BA_OK;
      }
    }
  }
  // The timed runs solve a short problem (at most 3 attempts) in place: the
  // caller passes scratch copies of the state.
  ba_settings probe = *s;
  probe.grad_tol = probe.step_tol = 0.0;   // every window runs every timed attempt
  probe.max_iters = std::min(s->max_iters, 3);
  if (probe.max_iters < 1) probe.max_iters = 1;
  ba_report* reports = nullptr;
  e = hipMalloc(&reports, sizeof(ba_report) * b->wins.size());
  if (e != hipSuccess) return set_error(BA_ERR_OOM, "autotune reports");
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  // time one configuration: best of two runs after one warm-up; +inf when it
  // does not fit (LDS or workspace)
  auto time_cfg = [&](const ba_launch_config& c, float* ms_out) -> ba_status {
    *ms_out = 1e30f;
    ba_status r = ba_set_launch_config(b, &c);
    if (r == BA_ERR_UNSUPPORTED || r == BA_ERR_INVALID_ARG) return BA_OK;
    if (r != BA_OK) return r;
    int which = 0;
    if (pick_config(b, probe.precision, &which) != BA_OK) return BA_OK;
    size_t need = 0;
    if ((r = ba_workspace_size(nullptr, b, &probe, &need)) != BA_OK) return r;
    if (need > ws_bytes) return BA_OK;
    for (int rep = 0; rep < 3; ++rep) {
      (void)hipEventRecord(e0, hs);
      r = ba_solve_batched(b, &probe, poses, points, obs_uv, obs_w, workspace, ws_bytes, reports, nullptr, stream);
      (void)hipEventRecord(e1, hs);
      if (r != BA_OK) return r;
      (void)hipEventSynchronize(e1);
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (rep > 0) *ms_out = std::min(*ms_out, ms);
    }
    return BA_OK;
  };
  // coordinate descent over the knobs, in this order: work-item size, tile
  // size, per-class work-item multipliers, class chains on side streams
  ba_launch_config best;
  (void)ba_get_launch(b, &best);
  best.tile_pairs = 0;
  best.class_streams = 1;
  for (int c = 0; c < kClasses; ++c) best.class_chunk_mult[c] = 1;
  float best_ms = 1e30f;
  auto consider = [&](const ba_launch_config& c) -> ba_status {
    float ms = 0;
    ba_status r = time_cfg(c, &ms);
    if (r == BA_OK && ms < best_ms) {
      best_ms = ms;
      best = c;
    }
    return r;
  };
  for (int chunk : {1024, 2048, 4096, 8192, 16384}) {
    ba_launch_config c = best;
    c.chunk_obs = chunk;
    if ((st = consider(c)) != BA_OK) break;
  }
  if (st == BA_OK) {
    ba_launch_config c = best;
    c.tile_pairs = kTileSmall;
    st = consider(c);
  }
  const int mults[][kClasses] = {{1, 1, 2, 2}, {2, 2, 1, 1}, {1, 1, 1, 2}, {2, 1, 1, 1}};
  for (const auto& m : mults) {
    if (st != BA_OK) break;
    ba_launch_config c = best;
    for (int k = 0; k < kClasses; ++k) c.class_chunk_mult[k] = m[k];
    st = consider(c);
  }
  if (st == BA_OK) {
    ba_launch_config c = best;
    c.class_streams = 0;
    st = consider(c);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(reports);
  if (st != BA_OK) return st;
  if (best_ms >= 1e30f) return set_error(BA_ERR_WORKSPACE_TOO_SMALL, "no launch shape fits the workspace");
  if ((st = ba_set_launch_config(b, &best)) != BA_OK) return st;
  if (cache) {
    std::ofstream outf(cache, std::ios::app);
    outf << key << " " << best.chunk_obs << " " << best.tile_pairs;
    for (int k = 0; k < kClasses; ++k) outf << " " << best.class_chunk_mult[k];
    outf << " " << best.class_streams << "\n";
  }
  if (chosen_chunk_obs) *chosen_chunk_obs = best.chunk_obs;
  return BA_OK;
}

}  // extern "C"
