/*
 * ba.h -- C ABI of the MI355X (gfx950) sliding-window sparse bundle adjuster.
 *
 * The library solves the local sparse bundle adjustment of the paper's 3D module
 * (cuVSLAM, Sec. 2.2, Eq. 2 and Eq. 3): given keyframe poses T^bw_i
 * (base-from-world), landmarks p^w_j, a rig of cameras with fixed
 * camera-from-base transforms T^cb_k and pinhole intrinsics, and 2D observations
 * o of landmark j by camera k at pose i, it minimises
 *
 *     F = 1/2 sum_o w_o rho( || pi(T^cb_k T^bw_i p^w_j) - o ||^2 )
 *
 * (rho = Huber kernel on the pixel residual, w_o = observation weight) with
 * Levenberg-Marquardt.  Each linear system is solved "poses first, then points"
 * through the Schur complement (the sentence after Eq. 3): per-landmark
 * elimination of the 3x3 point blocks, an FP64 Cholesky of the reduced camera
 * system, then point back-substitution.
 *
 * Conventions (all arrays row-major, all values FP64 at this boundary):
 *   pose / extrinsic  : 3x4 [R | t] (12 doubles), x_out = R x_in + t
 *   pose update       : left perturbation T <- Exp(xi) T, xi = (rho, phi)
 *   intrinsics        : fx, fy, cx, cy (4 doubles per camera)
 *   observation pixel : (u, v), residual r = pi(x_c) - (u, v)
 *   damping           : U_ii += lambda * max(diag, 1e-9), likewise V_jj
 *   attempt           : one solve + candidate evaluation; accepted iff the robust
 *                       cost strictly decreases (lambda /= down), else rejected
 *                       (lambda *= up); a solve that meets a non-positive pivot
 *                       or a candidate with a camera depth <= min_depth is a
 *                       rejected attempt.  Exactly max_iters attempts run.
 *
 * Ownership: the caller owns every device buffer and the workspace.  The
 * library owns plan handles (ba_window, ba_batch).  A plan's structure is
 * immutable after creation; its one mutable part is the launch shape, which
 * ba_set_launch and ba_autotune replace (with new launch tables, and possibly
 * a new workspace size: query ba_workspace_size again).  Once any call on a
 * plan has been captured into a HIP graph, the tables they replace are kept
 * until the plan is destroyed, so a graph captured earlier still replays the
 * shape it was captured with (with the workspace it was captured with).  A
 * plan may be used concurrently on different streams with different
 * workspaces; re-tuning it concurrently with a solve is not allowed.
 * ba_solve, ba_solve_batched and ba_adjoint allocate no device memory, never
 * synchronise the stream and never read device memory back to the host, so a
 * caller may capture them into a HIP graph.  Plan creation allocates device
 * memory for the plan's index arrays (on the current device).
 * Side streams: on a plan whose windows fall into two or more size classes of
 * the Schur kernel (up to 8, 16, 23 and 32 free poses), the first call that is
 * not under stream capture creates two streams (default priority) and three
 * events, kept until the plan is destroyed.  Every later call forks the work
 * of the two largest classes onto them from `stream` (a solve: their whole LM
 * loop; the adjoint: its one pass) and joins it back with events, so all
 * of the call's work is still ordered on `stream`, and a capture records the
 * fork and join.  Until then (or for a one-class plan) everything runs on
 * `stream`.  Calls on one plan from several streams share the side streams:
 * still correct, but their forked work waits for each other there.  While a
 * capture on one stream holds the side streams (from its fork until the
 * capture ends), a call of the same plan on another stream runs all of its
 * work on its own stream instead.
 *
 * Errors: every call returns ba_status.  Argument and structure errors are
 * detected on the host before any device work and return a negative status;
 * ba_last_error() gives a thread-local description.  Numerical outcomes of a
 * solve (Cholesky failures, rejected candidates, non-finite input) are written
 * to the device-resident ba_report of each window.
 *
 * Limits of this implementation (checked at plan creation):
 *   n_poses <= 64 per window, n_cams <= 32, free poses <= 32 per window
 *   (<= 29 in BA_FP64, whose reduced system takes the 160 KB of LDS; reported
 *   by ba_workspace_size and the solve calls as BA_ERR_UNSUPPORTED),
 *   every landmark observed from >= 2 distinct (pose, camera) views,
 *   observations per landmark <= 4096, < 2^30 observations per batch.
 */
#ifndef BA_H
#define BA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ba_window_s* ba_window;  /* plan of one window's structure */
typedef struct ba_batch_s* ba_batch;    /* plan of many windows, packed window-major */

typedef enum {
  BA_OK = 0,
  BA_ERR_INVALID_ARG = -1,          /* NULL pointer, index out of range, bad value */
  BA_ERR_OOM = -2,                  /* host or plan device allocation failed */
  BA_ERR_HIP = -3,                  /* a HIP runtime call failed */
  BA_ERR_WORKSPACE_TOO_SMALL = -4,  /* ws_bytes below ba_workspace_size() */
  BA_ERR_UNSUPPORTED = -5,          /* structure beyond the limits above */
  BA_ERR_STATE = -6                 /* handle not usable for this call (e.g. host-only) */
} ba_status;

typedef enum {
  BA_FP64 = 0,   /* every step in FP64 */
  BA_MIXED = 1   /* FP32 observation stream, Jacobians, Hessian blocks and Schur
                    products; FP64 pose/point state, camera-frame transform,
                    cost sums, acceptance test, damping of S and the reduced-camera
                    Cholesky */
} ba_precision;

/* flags of ba_window_create */
enum { BA_CREATE_HOST_ONLY = 1 };   /* build and validate the plan, no device upload */

typedef struct {
  int32_t max_iters;      /* LM attempts (accepted + rejected); >= 0 */
  int32_t precision;      /* ba_precision */
  double lambda_init;     /* initial damping, > 0 (e.g. 1e-3) */
  double lambda_up;       /* factor on rejection, > 1 (10) */
  double lambda_down;     /* divisor on acceptance, > 1 (10) */
  double lambda_min;      /* clamp, > 0 (1e-10) */
  double lambda_max;      /* clamp (1e10) */
  double huber_delta;     /* pixels; <= 0 selects plain least squares */
  double min_depth;       /* candidate rejected if any camera depth Z <= min_depth */
  /* Per-window freeze (0 = off: every window runs max_iters attempts).  A
   * frozen window runs no more attempts; each remaining one is traced with
   * status 3, not accepted, cost and lambda unchanged, and not counted in
   * ba_report.iters.  The launches stay the same (graph-capturable): a frozen
   * window's work items return at once.  Window solves only (ba_solve,
   * ba_solve_batched, ba_solve_noalloc, ba_map_solve); ba_vi_solve requires 0. */
  double grad_tol;        /* before an attempt: freeze when max(|b~|_inf, |g_l|_inf) <= grad_tol,
                             b~ the reduced camera system's right-hand side at the attempt's
                             damping, g_l the landmark gradient (never when a landmark block is
                             not positive definite); >= 0 */
  double step_tol;        /* after an accepted attempt: freeze when the step's max-norm (pose
                             tangents, point moves) <= step_tol; >= 0 */
} ba_settings;

/* Per-window outcome, written by the device at the end of a solve. */
typedef struct {
  double initial_cost;    /* F at the input state */
  double final_cost;      /* F at the output state */
  double final_lambda;
  int32_t iters;          /* attempts run (frozen ones excluded) */
  int32_t accepted;       /* accepted attempts */
  int32_t chol_failures;  /* attempts rejected by a non-positive pivot */
  int32_t depth_rejects;  /* attempts rejected by min_depth */
  int32_t status;         /* 0 = ok, 1 = non-finite input cost, 2 = bad indices (motion-only,
                             triangulation), 3 / 4: see ba_triangulate */
  int32_t reserved;
} ba_report;

/* One attempt of one window (optional per-attempt trace). */
typedef struct {
  double cost;            /* F before the attempt */
  double cand_cost;       /* F at the candidate; NaN when none was formed */
  double lambda;          /* damping used */
  int32_t accepted;
  int32_t status;         /* 0 = candidate formed, 1 = pivot failure, 2 = depth, 3 = frozen */
} ba_iter_trace;

/* Plan statistics (host side; usable without a device). */
typedef struct {
  int32_t n_poses, n_points, n_cams, n_free;
  int64_t n_obs, n_pairs;   /* pairs = distinct (pose, landmark) */
  int32_t n_tiles, n_chunks;
  int64_t schur_blocks;     /* sum over landmarks of P(P+1)/2, P = free pairs */
  int64_t n_free_pairs;     /* pairs whose pose is free */
} ba_plan_info;

/* Validate one window's structure and build its plan.
 *   obs_pose, obs_point : HOST, n_obs each, indices in [0, n_poses) / [0, n_points)
 *   obs_cam             : HOST, n_obs, in [0, n_cams); NULL -> camera 0
 *   pose_fixed          : HOST, n_poses bytes (nonzero = held fixed); NULL -> pose 0 fixed
 *   intrinsics          : HOST, n_cams x 4 (fx, fy, cx, cy), finite, fx, fy > 0
 *   extrinsics          : HOST, n_cams x 12 camera-from-base [R | t]; NULL -> identity
 *   flags               : 0 or BA_CREATE_HOST_ONLY
 * The arrays are copied; the caller may free them after the call.  The user's
 * observation order is kept at every later call (obs_uv, obs_w, gradients). */
ba_status ba_window_create(int32_t n_poses, int32_t n_points, int32_t n_cams, int64_t n_obs,
                           const int32_t* obs_pose, const int32_t* obs_point,
                           const int32_t* obs_cam, const uint8_t* pose_fixed,
                           const double* intrinsics, const double* extrinsics,
                           int32_t flags, ba_window* out);
void ba_window_destroy(ba_window w);
ba_status ba_window_info(ba_window w, ba_plan_info* info);

/* Copy of the plan's landmark-major observation order: perm[k] = user index of
 * the k-th observation in plan order (HOST, n_obs).  For tests of the plan. */
ba_status ba_window_order(ba_window w, int64_t* perm);

/* Pack windows into one batch (device upload).  Windows keep their order;
 * batched arrays are concatenated window-major: poses (sum n_poses x 12),
 * points (sum n_points x 3), observations (sum n_obs, each window in its own
 * user order).  The windows may be destroyed after the call. */
ba_status ba_batch_create(int32_t n_windows, const ba_window* windows, ba_batch* out);
void ba_batch_destroy(ba_batch b);
ba_status ba_batch_info(ba_batch b, int32_t window, ba_plan_info* info);

/* Bytes of workspace needed by ba_solve / ba_solve_batched / ba_adjoint for this
 * plan and precision.  Exactly one of w, b is non-NULL. */
ba_status ba_workspace_size(ba_window w, ba_batch b, const ba_settings* s, size_t* bytes);

/* Solve one window in place.
 *   poses   : DEVICE, n_poses x 12, in/out (fixed poses are left untouched)
 *   points  : DEVICE, n_points x 3, in/out
 *   obs_uv  : DEVICE, n_obs x 2 pixels, user order
 *   obs_w   : DEVICE, n_obs weights; NULL -> all 1
 *   workspace: DEVICE, >= ba_workspace_size bytes, 256-byte aligned
 *   report  : DEVICE, one ba_report
 *   trace   : DEVICE, max_iters ba_iter_trace, or NULL
 *   stream  : hipStream_t (NULL = default stream)
 * Enqueued on `stream`; returns before the device finishes. */
ba_status ba_solve(ba_window w, const ba_settings* s, double* poses, double* points,
                   const double* obs_uv, const double* obs_w, void* workspace,
                   size_t ws_bytes, ba_report* report, ba_iter_trace* trace, void* stream);

/* Doubles of one preintegrated IMU factor record (ba_vi_preintegrate). */
#define BA_VI_PREINT_DOUBLES 320

/* Largest workspace of ba_solve_noalloc, in bytes, per device (64 MiB). */
#define BA_NOALLOC_SCRATCH_BYTES (64u << 20)

/* ba_solve without a workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture that must not call hipMalloc,
 * tight serving loops, harnesses that forbid allocation.  The workspace is a
 * static device array of BA_NOALLOC_SCRATCH_BYTES that the library holds on
 * each device it runs on until the process ends; the call itself allocates
 * nothing (no hipMalloc, hipFree or allocating library routine).  The first
 * call on a device looks up that device's copy of the array.
 * Every call on one device shares its array, which keeps the last call's
 * contents: calls that overlap on one GPU (on different streams, or beside a
 * replay of a graph that captured this call) race and corrupt each other, so
 * order them on one stream.  Nothing in the array needs to start at zero (the
 * solve initialises what it reads).  Arguments, results and errors as
 * ba_solve; a window whose workspace (ba_workspace_size) exceeds the limit
 * returns BA_ERR_WORKSPACE_TOO_SMALL before any device work. */
ba_status ba_solve_noalloc(ba_window w, const ba_settings* s, double* poses, double* points,
                           const double* obs_uv, const double* obs_w, ba_report* report,
                           ba_iter_trace* trace, void* stream);

/* Solve every window of a batch in one launch sequence (one kernel per stage
 * and size class covering that class's windows; the classes run as concurrent
 * chains, see "Side streams" above).  Arrays are packed window-major (see
 * ba_batch_create);
 * reports: DEVICE, n_windows; traces: DEVICE, n_windows x max_iters or NULL.
 * Every window runs the same number of attempts. */
ba_status ba_solve_batched(ba_batch b, const ba_settings* s, double* poses, double* points,
                           const double* obs_uv, const double* obs_w, void* workspace,
                           size_t ws_bytes, ba_report* reports, ba_iter_trace* traces,
                           void* stream);

/* Implicit-function adjoint at a converged state x* (given, not recomputed).
 * With a = H*^-1 dL/dx (H* = exact Hessian of F over the free variables, no
 * damping) it writes, per observation in user order,
 *     grad_uv[o] = w_o (rho' I + 2 rho'' r r^T) J_o a,   grad_w[o] = -rho' r^T J_o a.
 *   grad_poses : DEVICE, n_poses x 12 ambient cotangent dL/d[R | t] (rows of
 *                fixed poses are ignored); mapped to the left-perturbation tangent
 *   grad_points: DEVICE, n_points x 3, or NULL (zero)
 *   grad_uv    : DEVICE out, n_obs x 2;  grad_w: DEVICE out, n_obs, or NULL
 *   reports    : DEVICE, per window; chol_failures = 1 when H* was not positive
 *                definite on the reduced camera system
 * Exactly one of w, b is non-NULL; with b the arrays are packed as in
 * ba_solve_batched.  settings->lambda_* and max_iters are ignored. */
ba_status ba_adjoint(ba_window w, ba_batch b, const ba_settings* s, const double* poses,
                     const double* points, const double* obs_uv, const double* obs_w,
                     const double* grad_poses, const double* grad_points, double* grad_uv,
                     double* grad_w, void* workspace, size_t ws_bytes, ba_report* reports,
                     void* stream);

/* Launch shape of a plan's batched solve (one launch per
 * stage and size class).  Defaults: chunk_obs from the plan's size,
 * tile_pairs 0, every class_chunk_mult 1, class_streams 1. */
typedef struct {
  int32_t chunk_obs;            /* target observations per work item, 128..65536 */
  int32_t tile_pairs;           /* pairs per tile: 0 = 256 when its LDS fits, else 64; or 64 / 256 */
  int32_t class_chunk_mult[4];  /* per size class (up to 8, 16, 23, 32 free poses): work items of
                                   about class_chunk_mult x chunk_obs observations, 1..4 */
  int32_t class_streams;        /* 1: the size classes run as concurrent chains on two side
                                   streams; 0: every launch on the call's stream */
} ba_launch_config;

/* Launch-shape tuning.  ba_autotune times candidate shapes of the batched
 * solve on this plan (3-attempt solves, best of two after a warm-up;
 * synchronises the stream; not capturable) by coordinate descent: chunk_obs
 * over 1024..16384, then 64-pair tiles, then four per-class multiplier sets,
 * then all classes on one stream; it keeps the fastest in the plan and
 * returns its chunk_obs (ba_get_launch gives the whole shape).  The state
 * arrays are modified: pass scratch copies.  Shapes whose workspace exceeds
 * ws_bytes are skipped.  Results are cached per (device name, precision,
 * window count, size bucket, largest window, windows and size bucket of each
 * size class) in the file named by $BA_TUNE_CACHE when that variable is set.
 * ba_set_launch sets chunk_obs (the other fields kept), ba_set_launch_config
 * the whole shape (INVALID_ARG outside the ranges above, before any change;
 * on a failed table upload the previous shape is rebuilt). */
ba_status ba_autotune(ba_batch b, const ba_settings* s, double* poses, double* points,
                      const double* obs_uv, const double* obs_w, void* workspace,
                      size_t ws_bytes, void* stream, int32_t* chosen_chunk_obs);
ba_status ba_set_launch(ba_batch b, int32_t chunk_obs);
ba_status ba_set_launch_config(ba_batch b, const ba_launch_config* cfg);
ba_status ba_get_launch(ba_batch b, ba_launch_config* cfg);

/* Diagnostics: the same solve as ba_solve_batched with HIP events recorded on
 * `stream` between the launches; writes the summed device time in ms of each
 * stage over all attempts: stage_ms[0] linearise + Schur (pass A),
 * [1] reduction + Cholesky + candidate poses, [2] back-substitution +
 * candidate cost (pass B), [3] acceptance.  Synchronises the stream; not
 * capturable.  For benchmarks and profiling only. */
ba_status ba_profile_stages(ba_batch b, const ba_settings* s, double* poses, double* points,
                            const double* obs_uv, const double* obs_w, void* workspace,
                            size_t ws_bytes, ba_report* reports, void* stream, double* stage_ms);

/* ---------------------------------------------------------------------------
 * Motion-only bundle adjustment (paper Sec. 2.2: the frame pose estimated from
 * 2D observations of landmarks taken from the local map, Eq. 4 for a stereo
 * pair, Eq. 6 for a multi-camera rig; Eq. 14, the loop-closure relative pose
 * against landmarks moved into a map frame by a known T^mw).  Each frame's pose
 * T minimises 1/2 sum_o w_o rho(|pi(T_cb_k T M p_j) - o|^2) over its own
 * observations, with the landmarks p_j FIXED (M = T^mw, or identity); the same
 * Huber kernel, left perturbation and LM schedule as ba_solve.
 * ------------------------------------------------------------------------- */

typedef struct ba_rig_s* ba_rig;   /* a camera rig resident on one device */

/* Upload a rig to the current device.
 *   intrinsics : HOST, n_cams x 4 (fx, fy, cx, cy), finite, fx, fy > 0
 *   extrinsics : HOST, n_cams x 12 camera-from-base [R | t]; NULL -> identity
 * 1 <= n_cams <= 32.  Errors: INVALID_ARG (bad values), UNSUPPORTED (> 32
 * cameras), OOM / HIP.  The library owns the handle; ba_rig_destroy frees it. */
ba_status ba_rig_create(int32_t n_cams, const double* intrinsics, const double* extrinsics,
                        ba_rig* out);
void ba_rig_destroy(ba_rig rig);

/* Waves of 64 lanes that share one frame in ba_pnp_solve on this rig: 1, 2 or
 * 4, or 0 (the default) to choose from the frame count and the mean
 * observations per frame.  Several waves per frame split its observations and
 * add their sums in a fixed order, so results differ from one wave per frame
 * only by rounding.  Errors: INVALID_ARG (NULL rig or another value). */
ba_status ba_rig_set_waves_per_frame(ba_rig rig, int32_t waves_per_frame);

/* Refine n_frames independent poses: exactly s->max_iters LM attempts each.
 * Every array is DEVICE memory on the rig's device:
 *   frame_obs_begin : n_frames + 1 int32; frame f owns observations
 *                     [frame_obs_begin[f], frame_obs_begin[f + 1]) (non-decreasing,
 *                     within [0, n_obs])
 *   poses           : n_frames x 12 [R | t], row-major, in/out (base-from-world,
 *                     or base-from-map when frame_transform is given)
 *   points          : n_points x 3 landmarks (world frame), read only
 *   obs_point       : n_obs int32 in [0, n_points)
 *   obs_cam         : n_obs int32 in [0, n_cams); NULL -> camera 0
 *   obs_uv          : n_obs x 2 pixels
 *   obs_w           : n_obs weights; NULL -> all 1
 *   frame_transform : n_frames x 12 T^mw applied to the landmarks; NULL -> none
 *   reports         : n_frames ba_report; NULL -> not written
 *   traces          : n_frames x max_iters ba_iter_trace (frame-major); may be NULL
 * s->precision: BA_MIXED accumulates the 6x6 blocks in FP32 per lane (FP64 sums
 * across lanes, FP64 Cholesky, acceptance and pose); BA_FP64 throughout.
 * Host checks return INVALID_ARG / UNSUPPORTED before any device work.  A frame
 * whose observation range or indices are out of range is left unchanged with
 * report status 2.  Allocates nothing and does not synchronise (capturable). */
ba_status ba_pnp_solve(ba_rig rig, const ba_settings* s, int32_t n_frames, int64_t n_obs,
                       int64_t n_points, const int32_t* frame_obs_begin, double* poses,
                       const double* points, const int32_t* obs_point, const int32_t* obs_cam,
                       const double* obs_uv, const double* obs_w, const double* frame_transform,
                       ba_report* reports, ba_iter_trace* traces, void* stream);

/* -------------------------------------------------------------------------
 * Multi-view triangulation (paper Sec. 2.2, 3D module: new landmarks are
 * triangulated from the multi-view observations of a keyframe before they
 * enter the local map).  Each landmark j is estimated from its own
 * observations with the poses FIXED: first the weighted least-squares
 * intersection of the viewing rays, (sum_o w_o (I - d_o d_o^T)) p0 =
 * sum_o w_o (I - d_o d_o^T) c_o (c_o the camera centre, d_o the unit ray through
 * the pixel, world frame), then exactly s->max_iters LM attempts on
 * 1/2 sum_o w_o rho(|pi(T_cb_k T_bw_i p) - o|^2) over p alone, with the Huber
 * kernel, damping, depth guard and acceptance of ba_solve.
 * ------------------------------------------------------------------------- */

/* Every array is DEVICE memory on the rig's device:
 *   point_obs_begin : n_points + 1 int32; landmark j owns observations
 *                     [point_obs_begin[j], point_obs_begin[j + 1]) (within [0, n_obs])
 *   poses           : n_poses x 12 [R | t] base-from-world, row-major, read only
 *   obs_pose        : n_obs int32 in [0, n_poses)
 *   obs_cam         : n_obs int32 in [0, n_cams); NULL -> camera 0
 *   obs_uv          : n_obs x 2 pixels
 *   obs_w           : n_obs weights; NULL -> all 1
 *   points          : n_points x 3, written: the refined landmark (status 0), the
 *                     unrefined ray intersection (status 4), NaN (status 2, 3)
 *   reports         : n_points ba_report or NULL; status 0 ok, 1 non-finite
 *                     start cost, 2 observation range or index out of range,
 *                     3 degenerate (fewer than two observations, or a Cholesky
 *                     pivot of the ray system <= 1e-10 times its trace), 4 the
 *                     start is at depth <= min_depth in one of its views
 *                     (costs NaN and no attempts for 2-4)
 *   traces          : n_points x max_iters ba_iter_trace (landmark-major) or NULL
 * s->precision: BA_MIXED accumulates V and g in FP32 (FP64 transform, residual,
 * cost, Cholesky and point); BA_FP64 throughout.  Host checks return
 * INVALID_ARG / UNSUPPORTED before any device work.  Allocates nothing and does
 * not synchronise (capturable). */
ba_status ba_triangulate(ba_rig rig, const ba_settings* s, int32_t n_points, int64_t n_obs,
                         int32_t n_poses, const int32_t* point_obs_begin, const double* poses,
                         const int32_t* obs_pose, const int32_t* obs_cam, const double* obs_uv,
                         const double* obs_w, double* points, ba_report* reports,
                         ba_iter_trace* traces, void* stream);

/* -------------------------------------------------------------------------
 * Pose-graph optimisation (paper Sec. 2.3, Eq. 15): keyframe poses T_i
 * (WORLD-from-base here, so that T_i^-1 T_j is the pose of base j in base i)
 * minimise 1/2 sum_e w_e |Log(D_ij^-1 T_i^-1 T_j)|^2 over the graph's edges,
 * with D_ij the measured pose deltas (integrated frontend predictions or loop
 * closures) and Log the SE(3) logarithm, xi = (rho, phi).  Poses flagged fixed
 * are held.  Exactly s->max_iters LM attempts with the damping, Cholesky-failure
 * and strict-decrease rules of ba_solve (left perturbation T <- Exp(xi) T);
 * the linear systems are solved by a sparse block Cholesky ordered by nested
 * dissection.  Always FP64 (s->precision is ignored); huber_delta and
 * min_depth do not apply.
 * ------------------------------------------------------------------------- */

typedef struct ba_graph_s* ba_graph;   /* a pose graph's structure on one device */

/* Plan a graph: edge e joins poses edge_i[e] and edge_j[e] (HOST arrays, n_edges
 * each, indices in [0, n_poses), edge_i != edge_j); pose_fixed: HOST, n_poses,
 * NULL -> pose 0 fixed.  Orders the free poses, computes the factor's pattern
 * and uploads the plan to the current device (flags BA_CREATE_HOST_ONLY: host
 * plan only, for ba_graph_info / ba_graph_plan_array; such a handle cannot
 * solve).  Errors: INVALID_ARG (bad indices, sizes or flags), OOM / HIP.  The
 * library owns the handle; ba_graph_destroy frees it. */
ba_status ba_graph_create(int32_t n_poses, int32_t n_edges, const int32_t* edge_i,
                          const int32_t* edge_j, const uint8_t* pose_fixed, int32_t flags,
                          ba_graph* out);

/* Host view of one plan table (for inspection and tests; valid while the
 * handle lives): which = 0 col_of_pose, 1 pose_of_col, 2 lev_ptr, 3 blk_ptr,
 * 4 blk_row, 5 upd_ptr, 6 upd_a, 7 upd_b, 8 fwd_ptr, 9 fwd_blk, 10 fwd_col,
 * 11 asm_ptr, 12 asm_edge, 13 rhs_ptr, 14 rhs_edge.  Columns are in
 * elimination order grouped by level; a column's blocks are its diagonal block
 * then its off-diagonal blocks by increasing row; block b of the update list
 * of target t contributes L_{upd_a} L_{upd_b}^T; asm/rhs entries are 2 e + s
 * (s = 1: subtracted).  Errors: INVALID_ARG. */
ba_status ba_graph_plan_array(ba_graph g, int32_t which, const int32_t** data, int64_t* len);
void ba_graph_destroy(ba_graph g);

/* Free poses, levels of the elimination tree and 6x6 blocks of the factor (any
 * output may be NULL).  Errors: INVALID_ARG (NULL graph). */
ba_status ba_graph_info(ba_graph g, int32_t* n_free, int32_t* n_levels, int32_t* n_blocks);

/* Workspace bytes ba_pgo_solve needs for this graph.  Errors: INVALID_ARG. */
ba_status ba_graph_workspace_size(ba_graph g, size_t* bytes);

/* Solve in place.  DEVICE arrays on the graph's device:
 *   poses     : n_poses x 12 [R | t] world-from-base, row-major, in/out
 *   deltas    : n_edges x 12 [R | t] measured D_ij (pose of base j in base i)
 *   edge_w    : n_edges weights, or NULL (all 1)
 *   workspace : >= ba_graph_workspace_size bytes, 256-byte aligned, caller-owned
 *   report    : 1 ba_report or NULL; traces: max_iters ba_iter_trace or NULL
 * Errors: INVALID_ARG, WORKSPACE_TOO_SMALL, STATE (host-only handle), HIP.
 * Allocates nothing and does not synchronise (capturable); calls that share a
 * workspace must be ordered on one stream. */
ba_status ba_pgo_solve(ba_graph g, const ba_settings* s, double* poses, const double* deltas,
                       const double* edge_w, void* workspace, size_t ws_bytes, ba_report* report,
                       ba_iter_trace* traces, void* stream);

/* -------------------------------------------------------------------------
 * Visual-inertial window solve (paper Sec. 2.2, "Visual-Inertial", Eq. 9):
 * the state of keyframe i is S_i = [T_i, v_i, b^a_i, b^w_i] (pose, world-frame
 * velocity of the base, accelerometer and gyroscope biases), consecutive
 * states are tied by an IMU factor (on-manifold preintegration of the IMU
 * samples between them, after Forster et al. 2017, which the paper follows),
 * and the window minimises the IMU factors plus the visual cost of ba_solve.
 * The IMU frame is the base frame.  IMU terms are FP64 in both precisions.
 * ------------------------------------------------------------------------- */

/* Preintegrate the samples of n_factors keyframe intervals.  DEVICE arrays:
 * sample_begin (n_factors + 1): interval f owns samples [sample_begin[f],
 * sample_begin[f + 1]); gyro, accel (n_samples x 3): angular rate (rad/s) and
 * specific force (m/s^2) of each sample, constant over dt seconds; bias_bar
 * (n_factors x 6: b^a then b^w) the bias estimates to integrate at; preint
 * (n_factors x BA_VI_PREINT_DOUBLES) out.  noise: HOST 4 densities sigma_g
 * (rad/s/sqrt(Hz)), sigma_a (m/s^2/sqrt(Hz)), sigma_bg, sigma_ba (bias random
 * walks) for the information of each factor.  An interval needs at least two
 * samples: the covariance of one sample is singular, and an interval of fewer
 * samples gets NaN information (a solve with it reports status 1, non-finite
 * cost).  One thread per interval; allocates nothing.  Errors: INVALID_ARG. */
ba_status ba_vi_preintegrate(int32_t n_factors, const int32_t* sample_begin, const double* gyro,
                             const double* accel, double dt, const double* bias_bar, const double* noise,
                             double* preint, void* stream);

/* Workspace of ba_vi_solve (2 <= n_poses <= 24).  Errors: as ba_workspace_size,
 * UNSUPPORTED for other pose counts. */
ba_status ba_vi_workspace_size(ba_window w, const ba_settings* s, size_t* bytes);

/* ba_solve of one window with the IMU factors between its consecutive poses
 * (pose f and f + 1, factor f of preint, n_poses - 1 records from
 * ba_vi_preintegrate).  gravity: HOST 3, world frame (m/s^2).  states: DEVICE
 * n_poses x 9 (v, b^a, b^w), in/out; every state's velocity and biases are
 * free (the window's fixed poses stay fixed).  Other arguments as ba_solve.
 * Per attempt the IMU factors are linearised at the current state and their
 * velocities and biases are eliminated onto the poses before the reduced
 * camera system is solved.  Errors: as ba_solve, UNSUPPORTED (pose count). */
ba_status ba_vi_solve(ba_window w, const ba_settings* s, const double* preint, const double* gravity,
                      double* poses, double* points, double* states, const double* obs_uv, const double* obs_w,
                      void* workspace, size_t ws_bytes, ba_report* report, ba_iter_trace* trace, void* stream);

/* -------------------------------------------------------------------------
 * Sliding-window local map (paper Sec. 2.1: the frontend keeps the last N
 * keyframe poses with the landmarks visible from them and their
 * observations; Sec. 2.2: at a keyframe, triangulated landmarks enter the map
 * with their observations and the sparse bundle adjustment refines it).
 * Rules (the paper gives none):
 *   - inserting a keyframe into a full map (max_keyframes) first drops the
 *     oldest keyframe with all its observations, then every landmark left
 *     with fewer than two distinct (keyframe, camera) views, with its
 *     remaining observations (no marginalisation);
 *   - an insertion brings the keyframe's pose, the landmarks created at it
 *     (caller ids and positions) and observations; each observation names a
 *     keyframe of the window after the insertion (0 = oldest), so a new
 *     landmark may also be seen in earlier keyframes;
 *   - every new landmark needs two distinct views; ids are unique in the map;
 *     an invalid insertion returns INVALID_ARG and leaves the map unchanged;
 *   - the solver's window: keyframes oldest first with the oldest fixed,
 *     landmarks in order of creation, observations in order of insertion.
 * Values (poses, points, pixels, weights) live on the map's device in the
 * window's order, so a solve refines them in place and the next insertion
 * carries the refined values over.  Not thread-safe: calls on one map must be
 * ordered by the caller.
 * ------------------------------------------------------------------------- */
typedef struct ba_map_s* ba_map;

/* n_cams cameras (intrinsics HOST n_cams x 4, extrinsics HOST n_cams x 12 or
 * NULL, as ba_window_create); 2 <= max_keyframes <= 64; flags 0 or
 * BA_CREATE_HOST_ONLY (index lists only, no device values: for inspection).
 * The device is the current one.  Errors: INVALID_ARG. */
ba_status ba_map_create(int32_t max_keyframes, int32_t n_cams, const double* intrinsics,
                        const double* extrinsics, int32_t flags, ba_map* out);
void ba_map_destroy(ba_map m);

/* Insert a keyframe.  HOST arrays: pose (12, base-from-world), new_ids
 * (n_new), new_points (n_new x 3 world), obs_kf (n_obs, keyframe index in the
 * window after the insertion), obs_lm (n_obs landmark ids), obs_cam (n_obs or
 * NULL: camera 0), obs_uv (n_obs x 2), obs_w (n_obs or NULL: 1).  Writes the
 * number of landmarks the slide dropped to *n_dropped (may be NULL).  Device
 * work (staging copies and one gather kernel per array) runs on `stream`;
 * the call waits for it, and may allocate device memory when the window
 * grows.  Errors: INVALID_ARG (map unchanged), OOM, HIP. */
ba_status ba_map_add_keyframe(ba_map m, const double* pose, int32_t n_new, const int64_t* new_ids,
                              const double* new_points, int64_t n_obs, const int32_t* obs_kf,
                              const int64_t* obs_lm, const int32_t* obs_cam, const double* obs_uv,
                              const double* obs_w, int32_t* n_dropped, void* stream);

/* Sizes of the current window (any output may be NULL). */
ba_status ba_map_info(ba_map m, int32_t* n_keyframes, int32_t* n_points, int64_t* n_obs);

/* HOST copies of the window's index lists in the solver's layout (any may be
 * NULL; sized by ba_map_info): obs_pose, obs_point, obs_cam (int32, n_obs),
 * landmark_ids (int64, n_points). */
ba_status ba_map_lists(ba_map m, int32_t* obs_pose, int32_t* obs_point, int32_t* obs_cam,
                       int64_t* landmark_ids);

/* DEVICE arrays of the window's values, owned by the map and valid until the
 * next insertion or destroy: poses (n_keyframes x 12), points (n_points x 3),
 * obs_uv (n_obs x 2), obs_w (n_obs).  Errors: STATE for a host-only map. */
ba_status ba_map_arrays(ba_map m, double** poses, double** points, const double** obs_uv,
                        const double** obs_w);

/* HOST copies of the window's values (any may be NULL; sized by ba_map_info);
 * synchronous (waits for the device).  Errors: STATE for a host-only map. */
ba_status ba_map_read(ba_map m, double* poses, double* points, double* obs_uv, double* obs_w);

/* The plan of the current window (rebuilt after an insertion; owned by the
 * map, valid until the next insertion or destroy): for ba_workspace_size and
 * ba_solve.  Errors: STATE (fewer than two keyframes), as ba_window_create. */
ba_status ba_map_window(ba_map m, ba_window* window);

/* ba_solve of the current window on the map's device arrays, in place. */
ba_status ba_map_solve(ba_map m, const ba_settings* s, void* workspace, size_t ws_bytes,
                       ba_report* report, ba_iter_trace* trace, void* stream);

const char* ba_status_string(ba_status s);
const char* ba_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BA_H */
