// Sliding-window local map (include/ba.h, ba_map_*).
//
// Paper Sec. 2.1: the frontend keeps the last N keyframe poses with the
// landmarks visible from them and their observations; Sec. 2.2: at a new
// keyframe the triangulated landmarks enter the map with their observations
// and the sparse bundle adjustment refines it.  The window rules (drop the
// oldest keyframe of a full window with its observations, then every landmark
// left with fewer than two distinct (keyframe, camera) views) are stated in
// ba.h.
//
// The host keeps the index lists (which keyframe, landmark and camera each
// observation belongs to); the values (poses, points, pixels, weights) live
// on the device in the window's order, so refined estimates stay where the
// solver left them.  An insertion computes, on the host, where each row of
// the new window comes from (a row of the previous window, or the staging
// buffer of the insertion's new rows) and one gather kernel per array builds
// the new window; the plan of the window is rebuilt from the index lists
// (O(observations), no comparison sort) when a solve needs it.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/ba.h"

namespace ba {
ba_status set_error(ba_status s, const std::string& m);   // api.cpp: thread-local detail
}

namespace {

// Row r of `out` (R doubles) is row src[r] of `old`, or row -src[r] - 1 of
// `fresh` when src[r] < 0.
__global__ void k_map_gather(const double* old, const double* fresh, const int32_t* src, double* out, int n_rows,
                             int R) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)n_rows * R) return;
  const int row = (int)(i / R), c = (int)(i - (int64_t)row * R);
  const int s = src[row];
  out[i] = s >= 0 ? old[(int64_t)s * R + c] : fresh[(int64_t)(-s - 1) * R + c];
}

struct DevBuf {
  double* p = nullptr;
  size_t cap = 0;   // doubles
};

hipError_t ensure(DevBuf& b, size_t n) {
  if (b.cap >= n && b.p) return hipSuccess;
  if (b.p) {
    hipError_t e = hipFree(b.p);
    if (e != hipSuccess) return e;
    b.p = nullptr;
    b.cap = 0;
  }
  const size_t c = std::max<size_t>(n + n / 2, 64);
  hipError_t e = hipMalloc(&b.p, c * sizeof(double));
  if (e == hipSuccess) b.cap = c;
  return e;
}

}  // namespace

struct ba_map_s {
  int32_t max_kf = 0, n_cams = 0;
  bool host_only = false;
  int device = 0;
  std::vector<double> intrinsics, extrinsics;
  bool have_ext = false;
  // host index lists of the current window
  std::vector<int64_t> kf_serial;            // oldest first
  int64_t next_serial = 0;
  std::vector<int64_t> lm_id;                // landmark order (order of creation)
  std::vector<int64_t> ob_kf;                // per observation: keyframe serial
  std::vector<int64_t> ob_lm;                // landmark id
  std::vector<int32_t> ob_cam;
  bool any_weight = false;                   // some observation weight != 1
  // device values in window order (two buffers each, swapped per insertion)
  DevBuf poses[2], points[2], uv[2], w[2];
  int cur = 0;
  DevBuf stage;                              // new rows of an insertion
  int32_t* idx = nullptr;                    // gather sources
  size_t idx_cap = 0;
  // plan of the current window (rebuilt when the window changed)
  ba_window plan = nullptr;
  bool plan_dirty = true;
  std::mutex mu;
  ~ba_map_s() {
    if (plan) ba_window_destroy(plan);
    for (int k = 0; k < 2; ++k)
      for (DevBuf* b : {&poses[k], &points[k], &uv[k], &w[k]})
        if (b->p) (void)hipFree(b->p);
    if (stage.p) (void)hipFree(stage.p);
    if (idx) (void)hipFree(idx);
  }
};

namespace {

ba_status fail(ba_status s, const std::string& m) { return ba::set_error(s, m); }

ba_status hip_fail(hipError_t e, const char* what) {
  return fail(BA_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// The window's index lists in the solver's layout.
void window_lists(const ba_map_s& m, std::vector<int32_t>& op, std::vector<int32_t>& oj,
                  std::vector<int32_t>& oc) {
  std::unordered_map<int64_t, int32_t> kpos, lpos;
  for (size_t i = 0; i < m.kf_serial.size(); ++i) kpos[m.kf_serial[i]] = (int32_t)i;
  lpos.reserve(m.lm_id.size() * 2);
  for (size_t j = 0; j < m.lm_id.size(); ++j) lpos[m.lm_id[j]] = (int32_t)j;
  const size_t n = m.ob_kf.size();
  op.resize(n);
  oj.resize(n);
  oc.resize(n);
  for (size_t o = 0; o < n; ++o) {
    op[o] = kpos[m.ob_kf[o]];
    oj[o] = lpos[m.ob_lm[o]];
    oc[o] = m.ob_cam[o];
  }
}

}  // namespace

extern "C" {

ba_status ba_map_create(int32_t max_keyframes, int32_t n_cams, const double* intrinsics,
                        const double* extrinsics, int32_t flags, ba_map* out) {
  if (!out) return fail(BA_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (max_keyframes < 2 || max_keyframes > 64) return fail(BA_ERR_INVALID_ARG, "max_keyframes must be in [2, 64]");
  if (n_cams < 1 || n_cams > 32) return fail(BA_ERR_INVALID_ARG, "n_cams must be in [1, 32]");
  if (!intrinsics) return fail(BA_ERR_INVALID_ARG, "intrinsics is NULL");
  if (flags & ~BA_CREATE_HOST_ONLY) return fail(BA_ERR_INVALID_ARG, "unknown flags");
  ba_map_s* m = new ba_map_s();
  m->max_kf = max_keyframes;
  m->n_cams = n_cams;
  m->host_only = (flags & BA_CREATE_HOST_ONLY) != 0;
  m->intrinsics.assign(intrinsics, intrinsics + 4 * n_cams);
  if (extrinsics) {
    m->extrinsics.assign(extrinsics, extrinsics + 12 * n_cams);
    m->have_ext = true;
  }
  // the camera values are checked once by a plan of a two-keyframe window
  {
    const int32_t op[2] = {0, 1}, oj[2] = {0, 0};
    ba_window probe = nullptr;
    ba_status s = ba_window_create(2, 1, n_cams, 2, op, oj, nullptr, nullptr, intrinsics, extrinsics,
                                   BA_CREATE_HOST_ONLY, &probe);
    if (s != BA_OK) {
      delete m;
      return s;
    }
    ba_window_destroy(probe);
  }
  if (!m->host_only) {
    hipError_t e = hipGetDevice(&m->device);
    if (e != hipSuccess) {
      delete m;
      return hip_fail(e, "hipGetDevice");
    }
  }
  *out = m;
  return BA_OK;
}

void ba_map_destroy(ba_map m) { delete m; }

ba_status ba_map_add_keyframe(ba_map m, const double* pose, int32_t n_new, const int64_t* new_ids,
                              const double* new_points, int64_t n_obs, const int32_t* obs_kf,
                              const int64_t* obs_lm, const int32_t* obs_cam, const double* obs_uv,
                              const double* obs_w, int32_t* n_dropped, void* stream) {
  if (!m || !pose) return fail(BA_ERR_INVALID_ARG, "NULL map or pose");
  if (n_new < 0 || n_obs < 0) return fail(BA_ERR_INVALID_ARG, "negative count");
  if ((n_new > 0 && (!new_ids || !new_points)) || (n_obs > 0 && (!obs_kf || !obs_lm || !obs_uv)))
    return fail(BA_ERR_INVALID_ARG, "NULL array");
  std::lock_guard<std::mutex> lk(m->mu);
  for (int k = 0; k < 12; ++k)
    if (!std::isfinite(pose[k])) return fail(BA_ERR_INVALID_ARG, "non-finite pose");
  // ---- the slide, on copies
  const bool full = (int32_t)m->kf_serial.size() == m->max_kf;
  std::vector<int64_t> serials(m->kf_serial.begin() + (full ? 1 : 0), m->kf_serial.end());
  const int64_t serial = m->next_serial;
  serials.push_back(serial);
  const int64_t old = full ? m->kf_serial[0] : -1;
  const size_t n_old_obs = m->ob_kf.size(), n_old_lm = m->lm_id.size();
  std::vector<uint8_t> obs_keep(n_old_obs, 1);
  std::vector<uint8_t> lm_keep(n_old_lm, 1);
  std::unordered_map<int64_t, int32_t> lpos;
  lpos.reserve(n_old_lm * 2 + (size_t)n_new * 2);
  for (size_t j = 0; j < n_old_lm; ++j) lpos[m->lm_id[j]] = (int32_t)j;
  if (full) {
    // distinct (keyframe, camera) views per landmark after the oldest keyframe
    // leaves: views are counted up to two
    std::vector<int64_t> first_view(n_old_lm, -1);
    std::vector<uint8_t> nviews(n_old_lm, 0);
    for (size_t o = 0; o < n_old_obs; ++o) {
      if (m->ob_kf[o] == old) {
        obs_keep[o] = 0;
        continue;
      }
      const int32_t j = lpos[m->ob_lm[o]];
      const int64_t view = m->ob_kf[o] * 64 + m->ob_cam[o];
      if (nviews[j] == 0) {
        first_view[j] = view;
        nviews[j] = 1;
      } else if (nviews[j] == 1 && view != first_view[j]) {
        nviews[j] = 2;
      }
    }
    for (size_t j = 0; j < n_old_lm; ++j) lm_keep[j] = nviews[j] >= 2;
    for (size_t o = 0; o < n_old_obs; ++o)
      if (obs_keep[o] && !lm_keep[lpos[m->ob_lm[o]]]) obs_keep[o] = 0;
  }
  // ---- checks of the insertion against the window after the slide
  std::unordered_map<int64_t, int32_t> newpos;
  newpos.reserve((size_t)n_new * 2);
  for (int32_t k = 0; k < n_new; ++k) {
    auto it = lpos.find(new_ids[k]);
    if ((it != lpos.end() && lm_keep[it->second]) || !newpos.emplace(new_ids[k], k).second)
      return fail(BA_ERR_INVALID_ARG, "new landmark id repeated or already in the map");
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(new_points[3 * k + c])) return fail(BA_ERR_INVALID_ARG, "non-finite new landmark");
  }
  const int32_t n_kf = (int32_t)serials.size();
  std::vector<int64_t> new_first(n_new, -1);
  std::vector<uint8_t> new_views(n_new, 0);
  for (int64_t o = 0; o < n_obs; ++o) {
    if (obs_kf[o] < 0 || obs_kf[o] >= n_kf) return fail(BA_ERR_INVALID_ARG, "observation keyframe index out of range");
    const int32_t cam = obs_cam ? obs_cam[o] : 0;
    if (cam < 0 || cam >= m->n_cams) return fail(BA_ERR_INVALID_ARG, "observation camera out of range");
    if (!std::isfinite(obs_uv[2 * o]) || !std::isfinite(obs_uv[2 * o + 1]) || (obs_w && !std::isfinite(obs_w[o])))
      return fail(BA_ERR_INVALID_ARG, "non-finite observation");
    auto nit = newpos.find(obs_lm[o]);
    if (nit != newpos.end()) {
      const int32_t k = nit->second;
      const int64_t view = serials[obs_kf[o]] * 64 + cam;
      if (new_views[k] == 0) {
        new_first[k] = view;
        new_views[k] = 1;
      } else if (new_views[k] == 1 && view != new_first[k]) {
        new_views[k] = 2;
      }
      continue;
    }
    auto it = lpos.find(obs_lm[o]);
    if (it == lpos.end() || !lm_keep[it->second])
      return fail(BA_ERR_INVALID_ARG, "observation of a landmark not in the map");
  }
  for (int32_t k = 0; k < n_new; ++k)
    if (new_views[k] < 2) return fail(BA_ERR_INVALID_ARG, "new landmark with fewer than two distinct views");

  // ---- gather sources of the new window
  std::vector<int32_t> src_pose, src_lm, src_obs;
  for (size_t i = full ? 1 : 0; i < m->kf_serial.size(); ++i) src_pose.push_back((int32_t)i);
  src_pose.push_back(-1);
  for (size_t j = 0; j < n_old_lm; ++j)
    if (lm_keep[j]) src_lm.push_back((int32_t)j);
  for (int32_t k = 0; k < n_new; ++k) src_lm.push_back(-1 - k);
  for (size_t o = 0; o < n_old_obs; ++o)
    if (obs_keep[o]) src_obs.push_back((int32_t)o);
  for (int64_t o = 0; o < n_obs; ++o) src_obs.push_back((int32_t)(-1 - o));
  const int32_t dropped = (int32_t)(n_old_lm - std::count(lm_keep.begin(), lm_keep.end(), 1));

  // ---- device: the new window's values
  if (!m->host_only) {
    int cur_dev = 0;
    hipError_t e = hipGetDevice(&cur_dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if ((e = hipSetDevice(m->device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t st = (hipStream_t)stream;
    const int nxt = m->cur ^ 1;
    // staging: pose (12), new points (3 n_new), pixels (2 n_obs), weights (n_obs)
    const size_t o_pose = 0, o_pts = 12, o_uv = o_pts + 3 * (size_t)n_new, o_w = o_uv + 2 * (size_t)n_obs;
    const size_t n_stage = o_w + (size_t)n_obs;
    std::vector<double> hs(n_stage);
    std::memcpy(hs.data() + o_pose, pose, 12 * sizeof(double));
    if (n_new) std::memcpy(hs.data() + o_pts, new_points, 3 * (size_t)n_new * sizeof(double));
    if (n_obs) std::memcpy(hs.data() + o_uv, obs_uv, 2 * (size_t)n_obs * sizeof(double));
    for (int64_t o = 0; o < n_obs; ++o) hs[o_w + o] = obs_w ? obs_w[o] : 1.0;
    const size_t n_idx = src_pose.size() + src_lm.size() + src_obs.size();
    std::vector<int32_t> hi;
    hi.reserve(n_idx);
    hi.insert(hi.end(), src_pose.begin(), src_pose.end());
    hi.insert(hi.end(), src_lm.begin(), src_lm.end());
    hi.insert(hi.end(), src_obs.begin(), src_obs.end());
    if ((e = ensure(m->stage, n_stage)) != hipSuccess ||
        (e = ensure(m->poses[nxt], 12 * src_pose.size())) != hipSuccess ||
        (e = ensure(m->points[nxt], 3 * std::max<size_t>(src_lm.size(), 1))) != hipSuccess ||
        (e = ensure(m->uv[nxt], 2 * std::max<size_t>(src_obs.size(), 1))) != hipSuccess ||
        (e = ensure(m->w[nxt], std::max<size_t>(src_obs.size(), 1))) != hipSuccess) {
      (void)hipSetDevice(cur_dev);
      return fail(BA_ERR_OOM, "map buffers: hipMalloc failed");
    }
    if (m->idx_cap < n_idx) {
      if (m->idx) (void)hipFree(m->idx);
      m->idx = nullptr;
      m->idx_cap = 0;
      const size_t c = n_idx + n_idx / 2 + 64;
      if ((e = hipMalloc(&m->idx, c * sizeof(int32_t))) != hipSuccess) {
        (void)hipSetDevice(cur_dev);
        return fail(BA_ERR_OOM, "map index buffer: hipMalloc failed");
      }
      m->idx_cap = c;
    }
    e = hipMemcpyAsync(m->stage.p, hs.data(), n_stage * sizeof(double), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(m->idx, hi.data(), n_idx * sizeof(int32_t), hipMemcpyHostToDevice, st);
    const int32_t* ip = m->idx;
    const int32_t* il = ip + src_pose.size();
    const int32_t* io = il + src_lm.size();
    auto gather = [&](const DevBuf& from, const double* fresh, const int32_t* src, size_t rows, int R,
                      DevBuf& to) {
      if (rows == 0 || e != hipSuccess) return;
      const int64_t n = (int64_t)rows * R;
      hipLaunchKernelGGL(k_map_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, from.p, fresh, src,
                         to.p, (int)rows, R);
      e = hipGetLastError();
    };
    gather(m->poses[m->cur], m->stage.p + o_pose, ip, src_pose.size(), 12, m->poses[nxt]);
    gather(m->points[m->cur], m->stage.p + o_pts, il, src_lm.size(), 3, m->points[nxt]);
    gather(m->uv[m->cur], m->stage.p + o_uv, io, src_obs.size(), 2, m->uv[nxt]);
    gather(m->w[m->cur], m->stage.p + o_w, io, src_obs.size(), 1, m->w[nxt]);
    // the host staging vectors die here: wait for the copies
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipSetDevice(cur_dev);
    if (e != hipSuccess) return hip_fail(e, "map insertion");
    m->cur = nxt;
  }

  // ---- commit the host lists
  std::vector<int64_t> lm2, okf2, olm2;
  std::vector<int32_t> oc2;
  lm2.reserve(src_lm.size());
  for (size_t j = 0; j < n_old_lm; ++j)
    if (lm_keep[j]) lm2.push_back(m->lm_id[j]);
  for (int32_t k = 0; k < n_new; ++k) lm2.push_back(new_ids[k]);
  okf2.reserve(src_obs.size());
  olm2.reserve(src_obs.size());
  oc2.reserve(src_obs.size());
  bool anyw = false;
  for (size_t o = 0; o < n_old_obs; ++o)
    if (obs_keep[o]) {
      okf2.push_back(m->ob_kf[o]);
      olm2.push_back(m->ob_lm[o]);
      oc2.push_back(m->ob_cam[o]);
    }
  for (int64_t o = 0; o < n_obs; ++o) {
    okf2.push_back(serials[obs_kf[o]]);
    olm2.push_back(obs_lm[o]);
    oc2.push_back(obs_cam ? obs_cam[o] : 0);
    if (obs_w && obs_w[o] != 1.0) anyw = true;
  }
  m->kf_serial = std::move(serials);
  m->next_serial = serial + 1;
  m->lm_id = std::move(lm2);
  m->ob_kf = std::move(okf2);
  m->ob_lm = std::move(olm2);
  m->ob_cam = std::move(oc2);
  m->any_weight = m->any_weight || anyw;
  m->plan_dirty = true;
  if (n_dropped) *n_dropped = dropped;
  return BA_OK;
}

ba_status ba_map_info(ba_map m, int32_t* n_keyframes, int32_t* n_points, int64_t* n_obs) {
  if (!m) return fail(BA_ERR_INVALID_ARG, "map is NULL");
  std::lock_guard<std::mutex> lk(m->mu);
  if (n_keyframes) *n_keyframes = (int32_t)m->kf_serial.size();
  if (n_points) *n_points = (int32_t)m->lm_id.size();
  if (n_obs) *n_obs = (int64_t)m->ob_kf.size();
  return BA_OK;
}

ba_status ba_map_lists(ba_map m, int32_t* obs_pose, int32_t* obs_point, int32_t* obs_cam, int64_t* landmark_ids) {
  if (!m) return fail(BA_ERR_INVALID_ARG, "map is NULL");
  std::lock_guard<std::mutex> lk(m->mu);
  std::vector<int32_t> op, oj, oc;
  window_lists(*m, op, oj, oc);
  if (obs_pose) std::copy(op.begin(), op.end(), obs_pose);
  if (obs_point) std::copy(oj.begin(), oj.end(), obs_point);
  if (obs_cam) std::copy(oc.begin(), oc.end(), obs_cam);
  if (landmark_ids) std::copy(m->lm_id.begin(), m->lm_id.end(), landmark_ids);
  return BA_OK;
}

ba_status ba_map_arrays(ba_map m, double** poses, double** points, const double** obs_uv, const double** obs_w) {
  if (!m) return fail(BA_ERR_INVALID_ARG, "map is NULL");
  if (m->host_only) return fail(BA_ERR_STATE, "host-only map has no device arrays");
  std::lock_guard<std::mutex> lk(m->mu);
  if (poses) *poses = m->poses[m->cur].p;
  if (points) *points = m->points[m->cur].p;
  if (obs_uv) *obs_uv = m->uv[m->cur].p;
  if (obs_w) *obs_w = m->w[m->cur].p;
  return BA_OK;
}

ba_status ba_map_read(ba_map m, double* poses, double* points, double* obs_uv, double* obs_w) {
  if (!m) return fail(BA_ERR_INVALID_ARG, "map is NULL");
  if (m->host_only) return fail(BA_ERR_STATE, "host-only map has no device arrays");
  std::lock_guard<std::mutex> lk(m->mu);
  int cur_dev = 0;
  hipError_t e = hipGetDevice(&cur_dev);
  if (e == hipSuccess) e = hipSetDevice(m->device);
  const size_t K = m->kf_serial.size(), M = m->lm_id.size(), n = m->ob_kf.size();
  if (e == hipSuccess && poses && K) e = hipMemcpy(poses, m->poses[m->cur].p, 12 * K * sizeof(double), hipMemcpyDeviceToHost);
  if (e == hipSuccess && points && M) e = hipMemcpy(points, m->points[m->cur].p, 3 * M * sizeof(double), hipMemcpyDeviceToHost);
  if (e == hipSuccess && obs_uv && n) e = hipMemcpy(obs_uv, m->uv[m->cur].p, 2 * n * sizeof(double), hipMemcpyDeviceToHost);
  if (e == hipSuccess && obs_w && n) e = hipMemcpy(obs_w, m->w[m->cur].p, n * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipSetDevice(cur_dev);
  if (e != hipSuccess) return hip_fail(e, "map read");
  return BA_OK;
}

ba_status ba_map_window(ba_map m, ba_window* window) {
  if (!m || !window) return fail(BA_ERR_INVALID_ARG, "NULL argument");
  std::lock_guard<std::mutex> lk(m->mu);
  if ((int32_t)m->kf_serial.size() < 2) return fail(BA_ERR_STATE, "the map holds fewer than two keyframes");
  if (m->plan_dirty || !m->plan) {
    std::vector<int32_t> op, oj, oc;
    window_lists(*m, op, oj, oc);
    const int32_t K = (int32_t)m->kf_serial.size();
    std::vector<uint8_t> fixed(K, 0);
    fixed[0] = 1;
    ba_window w = nullptr;
    int cur_dev = 0;
    if (!m->host_only) {
      hipError_t e = hipGetDevice(&cur_dev);
      if (e == hipSuccess) e = hipSetDevice(m->device);
      if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    }
    ba_status s = ba_window_create(K, (int32_t)m->lm_id.size(), m->n_cams, (int64_t)op.size(), op.data(), oj.data(),
                                   oc.data(), fixed.data(), m->intrinsics.data(),
                                   m->have_ext ? m->extrinsics.data() : nullptr,
                                   m->host_only ? BA_CREATE_HOST_ONLY : 0, &w);
    if (!m->host_only) (void)hipSetDevice(cur_dev);
    if (s != BA_OK) return s;
    if (m->plan) ba_window_destroy(m->plan);
    m->plan = w;
    m->plan_dirty = false;
  }
  *window = m->plan;
  return BA_OK;
}

ba_status ba_map_solve(ba_map m, const ba_settings* s, void* workspace, size_t ws_bytes, ba_report* report,
                       ba_iter_trace* trace, void* stream) {
  if (!m) return fail(BA_ERR_INVALID_ARG, "map is NULL");
  if (m->host_only) return fail(BA_ERR_STATE, "host-only map cannot be solved");
  ba_window w = nullptr;
  ba_status st = ba_map_window(m, &w);
  if (st != BA_OK) return st;
  std::lock_guard<std::mutex> lk(m->mu);
  return ba_solve(w, s, m->poses[m->cur].p, m->points[m->cur].p, m->uv[m->cur].p,
                  m->any_weight ? m->w[m->cur].p : nullptr, workspace, ws_bytes, report, trace, stream);
}

}  // extern "C"
