/*
 * exact_mppi.h -- C ABI of the MI355X (gfx950) library for one MPPI control
 * step with exact footprint signed distance.
 *
 * Paper: "EXACT-MPPI" (arXiv 2605.29663).  Section and equation names below
 * refer to that paper.
 *
 * Conventions for every entry point
 *   - Return value: MPPI_OK (0) on success, a negative MPPI_E_* code on
 *     failure.  mppi_last_error(ctx) then holds a human-readable message.
 *     On failure no output is guaranteed to be written.
 *   - Pointers whose name starts with "d" (dposes, dU, ...) are DEVICE
 *     pointers on the context's device; every other pointer is host memory.
 *   - The caller owns every pointer it passes; the library copies whatever
 *     it keeps (footprint, points) into buffers it owns.
 *   - All device work is ordered on the context's stream.  Calls return
 *     without waiting for the GPU, except where "synchronous" is stated.
 *   - A context is not thread-safe: calls on one context must not overlap.
 *   - Floating point is IEEE binary32 on the device.
 */
#ifndef EXACT_MPPI_H
#define EXACT_MPPI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPPI_API __attribute__((visibility("default")))

enum {
    MPPI_OK = 0,
    MPPI_E_ARG = -1,          /* invalid argument (NULL, negative size, bad enum) */
    MPPI_E_FOOTPRINT = -2,    /* footprint rejected (not simple, degenerate, non-finite) */
    MPPI_E_NO_FOOTPRINT = -3, /* the requested footprint kind was never set */
    MPPI_E_CAPACITY = -4,     /* size outside the supported range */
    MPPI_E_HIP = -5,          /* a HIP runtime call failed (message has hipGetErrorString) */
    MPPI_E_STATE = -6         /* call order violated (e.g. no points set) */
};

enum { MPPI_FP_POLYGON = 0, MPPI_FP_RECTS = 1 };

/* Motion models, Section "Robot Kinematic Models".  Controls per model:
 *   UNICYCLE  (v, omega)          nu = 2
 *   ACKERMANN (v, delta), wheelbase L     nu = 2
 *   OMNI      (v_x, v_y, omega)   nu = 3
 *   SPIN      (omega)             nu = 1
 *   PARALLEL  (v_para)            nu = 1                                     */
enum { MPPI_UNICYCLE = 0, MPPI_ACKERMANN = 1, MPPI_OMNI = 2, MPPI_SPIN = 3, MPPI_PARALLEL = 4 };

/* Capacities. */
#define MPPI_MAX_B 64        /* polygon vertices */
#define MPPI_MAX_R 32        /* rectangles in a cover */
#define MPPI_MAX_T 128       /* horizon */
#define MPPI_MAX_K (1 << 20) /* rollouts */
#define MPPI_MAX_PATH 64     /* guidance waypoints */

typedef struct mppi_ctx_s* mppi_ctx;

/* Parameters of one control cycle (Algorithm 1 "Params", plus the cost
 * forms the paper leaves open).  Field by field:
 *   K, T, nu, model   rollouts, horizon, control width, MPPI_* model
 *   footprint_kind    MPPI_FP_POLYGON or MPPI_FP_RECTS (Section
 *                     "Computational Footprint Representations")
 *   dt, lambda        Euler step and softmax temperature
 *   wheelbase         L of the Ackermann model
 *   sigma[c]          standard deviation of the Gaussian perturbation of
 *                     control channel c
 *   u_min, u_max      box the sampled control is clipped to; the update uses
 *                     the clipped perturbation eps_eff = u - U_h
 *   d_safe, w_coll, w_rep, w_inf   obstacle penalty, unsafe flag and
 *                     augmented cost (Section "Safety Penalties and
 *                     Trajectory Validation")
 *   w_goal, goal[2]   task term w_goal * |(x, y) - goal|
 *   w_path            path-following task term w_path * (distance of (x, y)
 *                     to the guidance polyline set by set_guidance; no term
 *                     while no guidance is set)
 *   w_ctrl[c]         control term sum_c w_ctrl[c] u_c^2
 *   state_offset      1: the (r, h) term scores the post-step state q_{h+1}
 *                     (moving points at time (h+1) dt); 0: the pre-step q_h
 *   validate          1: run Algorithm 1 step 4 (nominal re-rollout,
 *                     d >= d_safe check, hold-and-reset on failure);
 *                     0: always execute U_0 and shift                       */
typedef struct mppi_params {
    int32_t K, T, nu, model, footprint_kind;
    float dt, lambda, wheelbase;
    float sigma[3], u_min[3], u_max[3];
    float d_safe, w_coll, w_rep, w_inf, w_goal, w_ctrl[3];
    float goal[2];
    int32_t state_offset;
    int32_t validate;
    float w_path;
} mppi_params;

/* Graph mode (enable != 0): mppi_step calls without diagnostics (diag NULL)
 * replay a captured hipGraph of the whole step (a one-scene batch of this
 * context, see mppi_batch_create: bit-identical results, fewer launch
 * overheads, the persistent distance kernel).  The first step of a
 * parameter set builds the batch and autotunes its item size
 * (mppi_batch_autotune: about 70 launches of the distance pass); the graph
 * is rebuilt when the parameters change and re-planned when points or
 * footprint change.  With profiling on (mppi_set_profiling) the batch runs
 * eagerly and mppi_get_profile reports its distance pass.  The call first
 * waits for the context's stream.  Disabling frees it.                     */
MPPI_API int mppi_set_graph(mppi_ctx ctx, int enable);

/* Weak guidance (Section "Problem Statement": a waypoint sequence from an
 * upstream module; the task term's "path following"): host array of n
 * planning-frame waypoints (x0, y0, x1, y1, ...), copied synchronously into
 * the context.  The task term adds w_path * min over the polyline's segments
 * of the point-segment distance (one waypoint: the distance to it).
 * 0 <= n <= MPPI_MAX_PATH; n = 0 removes the guidance.  Non-finite values:
 * MPPI_E_ARG.  Takes effect from the next step, in batches too.             */
MPPI_API int set_guidance(mppi_ctx ctx, const float* host_xy, int n);

/* Point-cloud pre-processing (Section "Problem Statement": the obstacle set
 * is the local point cloud restricted to a task-relevant height band and
 * downsampled to a fixed budget N before rollout evaluation; the paper does
 * not name the downsampling method).  Reading implemented:
 *   a point (x, y, z) is kept if it is finite, z_min <= z <= z_max and its
 *   single-precision squared planar range to center, (x-cx)^2 + (y-cy)^2,
 *   is <= r_max^2; its voxel is (floor(x / voxel), floor(y / voxel));
 *   each occupied voxel is represented by its kept point of lowest index;
 *   if more than n_out voxels are occupied, the n_out representatives of
 *   smallest (squared range, index) are kept; the kept points are written in
 *   ascending input order, the remaining slots up to n_out get valid = 0
 *   (x = y = 0).
 * dxyz: device m x 3 floats (row-major x, y, z, planning frame).  dx, dy,
 * dvalid: device outputs of n_out entries, ready for set_points.  n_kept:
 * host, may be NULL (non-NULL makes the call synchronous).  Deterministic.
 * Limits: 0 <= m <= MPPI_MAX_CLOUD, 0 <= n_out <= MPPI_MAX_CLOUD, voxel > 0,
 * r_max > 0, z_min <= z_max, all finite, and (max(|cx|, |cy|) + r_max) /
 * voxel < 2^29; otherwise MPPI_E_ARG.  Workspace: about 40 bytes per input
 * point, kept by the context.                                              */
#define MPPI_MAX_CLOUD (1 << 20)
typedef struct mppi_cloud_params {
    float z_min, z_max, r_max, voxel;
    int32_t n_out;
} mppi_cloud_params;
MPPI_API int cloud_downsample(mppi_ctx ctx, const float* dxyz, int m, const float center[2],
                              const mppi_cloud_params* cp, float* dx, float* dy,
                              unsigned char* dvalid, int* n_kept);

/* Optional device outputs of mppi_step; any pointer may be NULL.
 *   d_min   K*T, row-major [r][h]: minimum signed distance over points
 *   argmin  K*T: caller's index of the point attaining d_min (-1 if none)
 *   J       K: augmented cost J~
 *   w       K: normalised weights omega
 *   poses   K*T*4: scored pose (x, y, cos theta, sin theta)
 *   eps     K*T*nu: clipped perturbation eps_eff
 *   u       K*T*nu: sampled (clipped) control
 *   U_upd   T*nu: nominal after the weighted update, before validation
 *   d_nom   T: minimum signed distance along the updated nominal
 *   J_nom   1: noise-free cost of the updated nominal, the sum over its
 *              validation rollout of the same per-step terms as J (task,
 *              control and obstacle terms; + w_inf if some d_nom < d_safe);
 *              NaN when validation is off                                   */
typedef struct mppi_diag {
    float* d_min;
    int32_t* argmin;
    float* J;
    float* w;
    float* poses;
    float* eps;
    float* u;
    float* U_upd;
    float* d_nom;
    float* J_nom;
} mppi_diag;

/* Create a context on HIP device `device`; work is issued on `hip_stream`
 * (a hipStream_t; NULL = the legacy default stream).  *out receives the
 * handle.  Errors: MPPI_E_ARG, MPPI_E_HIP.                                   */
MPPI_API int mppi_create(mppi_ctx* out, int device, void* hip_stream);

/* Release every buffer of the context (synchronises its stream). */
MPPI_API int mppi_destroy(mppi_ctx ctx);

/* Message of the last failed call on ctx (ctx may be NULL for failures of
 * mppi_create).  The string stays valid until the next call on ctx.          */
MPPI_API const char* mppi_last_error(mppi_ctx ctx);

/* Set the effective footprint (Section "Computational Footprint
 * Representations").  host points to host memory:
 *   MPPI_FP_POLYGON: count = B vertices, x0,y0,x1,y1,... (2B floats), the
 *     ordered cyclic vertex list of a simple polygon, either orientation,
 *     3 <= B <= MPPI_MAX_B.  Rejected (MPPI_E_FOOTPRINT): a non-finite
 *     value, a zero-length edge, |area| < 1e-12 m^2, or two non-adjacent
 *     edges that touch or cross.  Collinear vertices are allowed.
 *   MPPI_FP_RECTS: count = R rectangles, (c_x, c_y, s_x, s_y) each (4R
 *     floats; centre and half extents, Section "Orthogonal Footprints via
 *     Rectangle Covering"), 1 <= R <= MPPI_MAX_R, s_x, s_y > 0, finite.
 * Both kinds may be set; mppi_params.footprint_kind picks one per step.
 * The data are copied; the call is synchronous.                             */
MPPI_API int set_footprint(mppi_ctx ctx, int kind, const float* host, int count);

/* Host-only check of a footprint description, with the rules of
 * set_footprint (no device work, no context).  On rejection the reason is
 * written to msg (host buffer of msg_len bytes, may be NULL).  Returns
 * MPPI_OK, MPPI_E_FOOTPRINT, MPPI_E_CAPACITY or MPPI_E_ARG.                 */
MPPI_API int mppi_check_footprint(int kind, const float* host, int count, char* msg, int msg_len);

/* Set the obstacle set O = {o_i} (Section "Robot--Obstacle Signed
 * Distance") as device structure-of-arrays of n points in the planning
 * frame.  dvx, dvy (may be NULL: static points) give a constant velocity
 * per point; the point at time t is o_i + v_i t.  dvalid (may be NULL: all
 * valid) is the validity mask of Section "Batched Rollout and Distance
 * Computation": masked points never contribute.  Points with a non-finite
 * coordinate or velocity are treated as masked.  n may be 0.  The data are
 * copied (stream-ordered) into library buffers, so the caller may reuse its
 * arrays once the stream has passed this call.                              */
MPPI_API int set_points(mppi_ctx ctx, const float* dx, const float* dy, const float* dvx,
               const float* dvy, const unsigned char* dvalid, int n);

/* Signed distance of n body-frame query points to the polygon footprint:
 * d = sigma(p) min_b d_seg,b(p) (Section "Distance to General Simple
 * Polygonal Footprint"; sign from the crossing-number test).  dpx, dpy, dd:
 * device arrays of n floats.  Negative inside, positive outside.           */
MPPI_API int sdf_polygon(mppi_ctx ctx, const float* dpx, const float* dpy, int n, float* dd);

/* Signed distance of n body-frame points to the rectangle cover:
 * d = min_j ( |max(a_j, 0)| + min(max(a_jx, a_jy), 0) ), a_j = |p - c_j| - s_j
 * (Section "Distance to Orthogonal Footprints").  Same layout as above.     */
MPPI_API int sdf_rectcover(mppi_ctx ctx, const float* dpx, const float* dpy, int n, float* dd);

/* Minimum signed-distance matrix for given poses (Section "Batched Rollout
 * and Distance Computation"; Algorithm 1 step 2): for each of the K*T poses
 * (device float4 (x, y, cos theta, sin theta), row-major [r][h]) every valid
 * point is moved to time (h + state_offset) dt, transformed into that pose's
 * body frame (Section "Rollout-Frame Transformation") and evaluated against
 * the `kind` footprint; the minimum over points goes to dd_min[r*T + h]
 * (+inf when no point is valid).  dargmin (may be NULL) receives the index,
 * in the caller's point array, of the lowest-index point attaining it (-1
 * when none).                                                              */
MPPI_API int sdf_min_poses(mppi_ctx ctx, const float* dposes, int K, int T, float dt, int state_offset,
                  int kind, float* dd_min, int* dargmin);

/* sdf_min_poses for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation, arguments, layouts, stream ordering and results (bit
 * for bit) as sdf_min_poses, but its distance keys live in a fixed device
 * array of MPPI_NOALLOC_MAX_POSES entries that the library holds on every
 * device it runs on until the process ends (set up by mppi_create), so the
 * call allocates nothing; the caller still passes the poses and outputs.
 * K * T above MPPI_NOALLOC_MAX_POSES: MPPI_E_CAPACITY; K = 0 does nothing
 * (the output pointers may then be NULL).  Every call on one
 * device shares that device's array: calls whose work overlaps on one device
 * (two contexts on different streams, or two threads) race and corrupt each
 * other's results; order them on one stream or synchronise between them.  */
#define MPPI_NOALLOC_MAX_POSES (1 << 19)
MPPI_API int sdf_min_poses_noalloc(mppi_ctx ctx, const float* dposes, int K, int T, float dt,
                                   int state_offset, int kind, float* dd_min, int* dargmin);

/* Noise-free augmented cost of n given control sequences from q0 (host, 3
 * floats): each sequence (device dUseq, n*T*nu floats, sequence-major) is
 * clamped to the control box, rolled out without noise and scored exactly as
 * a sampled rollout of Algorithm 1 steps 1-2 is (J~ = sum over the horizon
 * of phi_task + phi_ctrl + phi_obs, + w_inf when a distance falls below
 * d_safe), against the footprint and points set.  dJ: device, n floats.
 * prm supplies the model, horizon, costs and control box; its K, sigma and
 * lambda are not used.  1 <= n <= MPPI_MAX_K (else MPPI_E_CAPACITY).
 * Stream-ordered on the context's stream, no host synchronisation.  The
 * cost of sequence U equals J~ of a one-rollout mppi_step around U with
 * zero noise.                                                               */
MPPI_API int mppi_sequence_costs(mppi_ctx ctx, const mppi_params* prm, const float* q0,
                                 const float* dUseq, int n, float* dJ);

/* Sampling and rollout only (Algorithm 1 step 1): K perturbed control
 * sequences around the nominal dU (device, T*nu row-major) and their Euler
 * rollouts from q0 (host, 3 floats).  Outputs (device, any may be NULL):
 * dposes K*T*4, deps K*T*nu (clipped perturbation), du K*T*nu (sampled
 * control).  The noise of (rollout r, step h) is the deterministic function
 * of (seed, step, r, h) described with mppi_step.                          */
MPPI_API int mppi_rollout(mppi_ctx ctx, const mppi_params* prm, const float* q0, const float* dU,
                 uint64_t seed, uint64_t step, float* dposes, float* deps, float* du);

/* One control cycle, Algorithm 1:
 *   1. eps_h^(r) = sigma * z with z standard normal from Philox4x64-10
 *      (counter (h, r, step, 0), key (seed, 0)) and Box-Muller; the sampled
 *      control is clipped to [u_min, u_max]; K Euler rollouts from q0.
 *   2. d_min over the points (set_points) against the footprint of
 *      prm->footprint_kind in every rollout body frame; costs J, unsafe flag
 *      chi and augmented cost J~ (Section "Safety Penalties and Trajectory
 *      Validation").
 *   3. beta = min J~, omega = softmax(-(J~ - beta)/lambda), U += sum omega eps.
 *   4. (prm->validate) re-roll the updated U, d_nom over the points; if every
 *      d_nom >= d_safe: u* = U_0 and U is shifted left (last entry
 *      repeated); otherwise u* = 0 and U = 0.
 * q0: host, 3 floats (x, y, theta).  dU: device T*nu, updated in place.
 * u_out: host, nu floats receiving u*.  valid_out (host, may be NULL)
 * receives 1 if the nominal passed validation.  diag may be NULL.
 * Synchronous: returns after u_out has been written.                       */
MPPI_API int mppi_step(mppi_ctx ctx, const mppi_params* prm, const float* q0, float* dU, uint64_t seed,
              uint64_t step, float* u_out, int* valid_out, const mppi_diag* diag);

/* Tile-shape autotuner for the fused transform + signed distance + min
 * stage of mppi_step: for prm's shape and the footprint and points currently
 * set, time every candidate (workgroup size in {64, 128, 256} poses, number of
 * point chunks) on one sampled step with HIP events (reps launches each) and
 * keep the fastest for this context; mppi_step then uses it whenever the
 * shape (kind, padded primitive count, moving points, K*T, N) matches.  With
 * prm->validate the point-chunk count of the validation pass (T poses) is
 * tuned the same way.  out_block / out_nchunk (host, may be NULL) receive
 * the sampled pass's choice.  Results do not depend on the choice
 * (bit-identical).  Synchronous.                                            */
MPPI_API int mppi_autotune(mppi_ctx ctx, const mppi_params* prm, int reps, int* out_block,
                           int* out_nchunk);

/* The autotuned tile table of a context as text, one line per shape:
 * "kind padded moving npose n block nchunk".  mppi_tune_get writes it to buf
 * (host, len bytes; error MPPI_E_CAPACITY if it does not fit), mppi_tune_set
 * adds the lines of text (host, NUL-terminated) to the context's table.     */
MPPI_API int mppi_tune_get(mppi_ctx ctx, char* buf, int len);
MPPI_API int mppi_tune_set(mppi_ctx ctx, const char* text);

/* Fix the tile shape of every fused signed-distance launch of this context
 * (block = poses per workgroup: 64, 128 or 256; nchunk = point chunks, >= 1);
 * block = 0 returns to the autotuned / default shapes.  Results are
 * bit-identical for every shape; this exists for tests and experiments.   */
MPPI_API int mppi_set_tiles(mppi_ctx ctx, int block, int nchunk);

/* Kernel timing of the fused transform + signed distance + min stage of
 * mppi_step (the dominant kernel), measured with HIP events recorded on the
 * context's stream right before and after that launch.  enable != 0 turns
 * recording on and resets the totals; enable == 0 turns it off.           */
MPPI_API int mppi_set_profiling(mppi_ctx ctx, int enable);

/* Totals since profiling was enabled: *ms = summed event time of the
 * signed-distance launches of the sampled rollouts, *launches = their count.
 * Synchronous.                                                             */
MPPI_API int mppi_get_profile(mppi_ctx ctx, double* ms, long long* launches);

/* ------------------------------------------------------------------------
 * Batched step: many independent scenes of uneven size in one launch
 * sequence.  Each scene is an existing context (its footprint and point set)
 * plus its own mppi_params (model, K, T, costs may all differ).  The
 * signed-distance stage of all scenes runs as one persistent kernel per
 * register class pulling (scene, pose tile, point chunk) items from a
 * longest-first queue; the whole cycle can be captured in one hipGraph and
 * replayed.  Each scene's outputs are bit-identical to mppi_step on that
 * scene's context with the same arguments.
 * ------------------------------------------------------------------------ */
typedef struct mppi_batch_s* mppi_batch;

/* Create a batch over n contexts (host array `scenes`, all on one device,
 * footprint and points already set) with per-scene parameters (host array
 * `prms`, copied).  Work runs on `hip_stream`, which must not be the legacy
 * NULL stream when graphs are used; NULL makes the batch create its own
 * non-blocking stream.  The contexts must outlive the batch.  Errors:
 * MPPI_E_ARG, MPPI_E_CAPACITY, MPPI_E_NO_FOOTPRINT, MPPI_E_HIP (message via
 * mppi_batch_last_error(NULL)).                                             */
MPPI_API int mppi_batch_create(mppi_batch* out, const mppi_ctx* scenes, const mppi_params* prms,
                               int n, void* hip_stream);
MPPI_API int mppi_batch_destroy(mppi_batch b);
MPPI_API const char* mppi_batch_last_error(mppi_batch b);

/* offsets (host, n+1 ints): scene s's nominal U_s (T_s x nu_s, row-major)
 * lives at dU + offsets[s] in the packed array mppi_step_batched takes.     */
MPPI_API int mppi_batch_u_offsets(mppi_batch b, int* offsets);

/* Re-plan after set_points / set_footprint on any of the batch's contexts
 * (a step refuses with MPPI_E_STATE until then).  Drops the captured graph. */
MPPI_API int mppi_batch_refresh(mppi_batch b);

/* One control cycle (Algorithm 1, as in mppi_step) of every scene.
 * q0: host n x 3.  dU: device packed nominals (see mppi_batch_u_offsets),
 * updated in place.  seeds, steps: host n.  u_out: host n x 3 (unused
 * channels 0).  valid_out: host n, may be NULL.  use_graph != 0 replays the
 * captured graph (captured on the first such call; arguments are refreshed
 * by a host-to-device copy inside the graph, so dU, q0, seeds and steps may
 * change between calls).  Synchronous.                                     */
MPPI_API int mppi_step_batched(mppi_batch b, const float* q0, float* dU, const uint64_t* seeds,
                               const uint64_t* steps, float* u_out, int* valid_out, int use_graph);

/* Tile autotuner of the batch: after a warm-up, times the persistent
 * signed-distance pass for queue items of 2^16 .. 2^26 point-primitive pairs
 * (reps launches each, HIP events, a forward and a backward sweep, the
 * faster of the two kept) and re-plans with the fastest.
 * *out_work_per_item (may be NULL) receives it.  Results do not depend on
 * the choice.  Synchronous.                                                 */
MPPI_API int mppi_batch_autotune(mppi_batch b, int reps, double* out_work_per_item);

/* Fix the queue item size: work_per_item point-primitive pairs per item
 * (at least 2^16 are used), or 0 for the default (2^22, shrunk for small
 * batches to about two rounds of resident workgroups).  Re-plans; results
 * do not depend on the size.  Errors: MPPI_E_ARG (negative, NaN, > 1e15). */
MPPI_API int mppi_batch_set_work(mppi_batch b, double work_per_item);

/* Size of the current plan: queue items of the sampled-rollout pass and of
 * the validation pass, and the pairs per item the plan uses.  Any pointer
 * may be NULL.                                                              */
MPPI_API int mppi_batch_info(mppi_batch b, long long* items_main, long long* items_validation,
                             double* work_per_item);

/* J_nom (see mppi_diag) of every scene from the last batched step: host n. */
MPPI_API int mppi_batch_nominal_costs(mppi_batch b, float* J_out);

/* Diagnostics of scene `scene` from the last batched (or hybrid) step, read
 * from the batch's workspaces into device buffers of `diag` (the layouts of
 * mppi_diag): d_min (decoded from the merged distance keys exactly as the
 * cost stage decodes them), poses, eps, J, U_upd, d_nom (NaN where
 * validation is off) and J_nom; each may be NULL.  argmin, w and u are not
 * kept by a batch and must be NULL (MPPI_E_ARG).  The workspaces hold the
 * last step until the next step, refresh, set_work or autotune of the batch
 * (MPPI_E_STATE when no step ran since the last plan).  Synchronous.       */
MPPI_API int mppi_batch_scene_diag(mppi_batch b, int scene, const mppi_diag* diag);

/* Timing of the sampled-rollout signed-distance pass (all persistent
 * launches of one step, HIP events on the batch's stream) over the eager
 * steps (use_graph = 0) run since profiling was enabled; graph replays are
 * not timed.  get: total milliseconds and number of timed steps.           */
MPPI_API int mppi_batch_set_profiling(mppi_batch b, int enable);
MPPI_API int mppi_batch_get_profile(mppi_batch b, double* ms, long long* launches);

/* ------------------------------------------------------------------------
 * Hybrid-mode cycle (Section "Extension to Hybrid-Mode Platforms",
 * Algorithm 2): one Algorithm-1 cycle per motion mode (each mode its own
 * rollout family and nominal sequence, the footprint and points shared),
 * all modes in one batched launch, then a device-side selection:
 *   Jbar_m = J_m + lambda_switch [m != m_prev] if mode m validated, else +inf,
 *   where J_m is the mode's J_nom (see mppi_diag);
 *   no mode validated -> safe stop: zero command, mode stays m_prev;
 *   m* = argmin Jbar (lowest index on ties), kept at m_prev while the
 *   cooldown tau_cool > 0; tau_cool <- cool_max after a switch, else
 *   max(tau_cool - 1, 0);
 *   command = mode m*'s executed command u* in that mode's own command
 *   layout (v, delta) / (v, omega) / (vx, vy, omega) / (omega) / (v_para),
 *   with the deadzone correction: translational modes scale the linear part
 *   (v, or (vx, vy)) up to v_min when noise_v < |v| < v_min; spin-in-place
 *   sets |omega| to w_min (sign kept) when noise_w < |omega| < w_min.
 * ------------------------------------------------------------------------ */
typedef struct mppi_hybrid_s* mppi_hybrid;

typedef struct mppi_hybrid_params {
    float lambda_switch;  /* switching penalty, >= 0                          */
    int32_t cool_max;     /* cooldown length after a switch (cycles), >= 0    */
    float v_min, w_min;   /* minimum executable speed / yaw rate, >= 0        */
    float noise_v, noise_w; /* below these magnitudes no correction is made   */
} mppi_hybrid_params;

enum { MPPI_MAX_MODES = 8 };

/* Create the mode set over context `scene` (footprint and points are read
 * from it at every step; it must outlive the hybrid object): modes[m] are
 * full Algorithm-1 parameter sets (host, copied; their `model` selects the
 * dynamics, each must have validate = 1).  1 <= n_modes <= MPPI_MAX_MODES.
 * Noise of mode m uses Philox stream word m.  Errors as mppi_batch_create
 * (message via mppi_hybrid_last_error(NULL)).                              */
MPPI_API int mppi_hybrid_create(mppi_hybrid* out, mppi_ctx scene, const mppi_params* modes,
                                int n_modes, void* hip_stream);
MPPI_API int mppi_hybrid_destroy(mppi_hybrid h);
MPPI_API const char* mppi_hybrid_last_error(mppi_hybrid h);
/* The underlying batch (for mppi_batch_u_offsets / refresh / autotune).   */
MPPI_API mppi_batch mppi_hybrid_batch(mppi_hybrid h);

/* One hybrid cycle.  q0: host 3.  dU: device packed per-mode nominals
 * (layout of mppi_batch_u_offsets), updated in place by each mode's cycle.
 * seed, step: as mppi_step.  m_prev, tau_cool: host in/out (the selected
 * mode and the new cooldown on return).  u_out: host 3 (unused channels 0).
 * stopped (may be NULL): 1 for a safe stop.  J_modes, valid_modes (host
 * n_modes each, may be NULL): each mode's J_m and validation flag.
 * use_graph as mppi_step_batched.  Synchronous.  Errors: MPPI_E_ARG
 * (m_prev out of range, negative cooldown or thresholds), MPPI_E_STATE,
 * MPPI_E_HIP.                                                              */
MPPI_API int mppi_hybrid_step(mppi_hybrid h, const float q0[3], float* dU, uint64_t seed,
                              uint64_t step, const mppi_hybrid_params* hp, int* m_prev,
                              int* tau_cool, float u_out[3], int* stopped, float* J_modes,
                              int* valid_modes, int use_graph);

/* ------------------------------------------------------------------------
 * Learned sampling proposal (not part of the paper's method, which is
 * training-free): a multilayer perceptron maps features of the current state
 * to the mean control sequence MPPI samples around.  Features (in_dim =
 * 64 + 2 + T*nu floats): 64 polar bins of the minimum range of the valid
 * obstacle points in the robot frame (bins of a pseudo-angle, 16 per
 * quadrant; range clipped at r_max, divided by r_max; empty bin = 1), the
 * goal in the robot frame divided by r_max, and the previous control
 * sequence scaled to [-1, 1] by the control box.  Network: in_dim -> hidden
 * -> hidden -> T*nu, exact-erf GELU, bf16 operands on the matrix cores with
 * fp32 accumulation, fp32 master weights.  Outputs are in the same [-1, 1]
 * control scaling.  Training: mean squared error, Adam (0.9, 0.999, 1e-8).
 * Parameter vector (fp32): W1[in][hidden], b1, W2[hidden][hidden], b2,
 * W3[hidden][T*nu], b3.  All calls are stream-ordered on the proposal's
 * stream unless stated otherwise.
 * ------------------------------------------------------------------------ */
typedef struct mppi_proposal_s* mppi_proposal;

/* Shape: horizon T, control width nu, hidden width, largest batch.  Weights
 * start at zero (set them with proposal_set_params or proposal_load).      */
MPPI_API int proposal_create(mppi_proposal* out, int device, void* hip_stream, int T, int nu,
                             int hidden, int max_batch);
MPPI_API int proposal_destroy(mppi_proposal p);
MPPI_API const char* proposal_last_error(mppi_proposal p);
MPPI_API long long proposal_num_params(mppi_proposal p);
MPPI_API int proposal_shape(mppi_proposal p, int* in_dim, int* hidden, int* out_dim);
/* Copy the flat fp32 parameter vector in / out (host, n = num_params);
 * set_params also resets the Adam state.  Synchronous.                     */
MPPI_API int proposal_set_params(mppi_proposal p, const float* host, long long n);
MPPI_API int proposal_get_params(mppi_proposal p, float* host, long long n);
/* Goal (prm->goal), control box (prm->u_min, u_max) and range clip used by
 * features, outputs and target normalisation.                              */
MPPI_API int proposal_set_scaling(mppi_proposal p, const mppi_params* prm, float r_max);
/* Features of M states (dq0: device M x 3 poses; dU_prev: device M x T x nu)
 * against the valid points of ctx, into dfeat (device M x in_dim).          */
MPPI_API int proposal_features(mppi_proposal p, mppi_ctx ctx, const float* dq0,
                               const float* dU_prev, int M, float* dfeat);
/* Network output (scaled units, device M x T*nu) of M feature rows.        */
MPPI_API int proposal_forward(mppi_proposal p, const float* dfeat, int M, float* dout);
/* Output mode.  scale = 0 (default): the output y is the sequence in
 * scaled units, u = mid + half y.  scale > 0 (residual mode): the output is
 * a correction of the previous sequence carried in the features,
 * u = mid + half (u_prev_scaled + scale y), so the network only encodes the
 * update (bf16 operands then round the correction, not the sequence).
 * Saved with the weights.                                                   */
MPPI_API int proposal_set_residual(mppi_proposal p, float scale);
/* Sampling mean: the output mapped back into the control box (device
 * M x T x nu), ready to be the nominal of mppi_step.                        */
MPPI_API int proposal_mean(mppi_proposal p, const float* dfeat, int M, float* dU);
/* Control sequences (device M x T x nu) -> training targets in the output's
 * units; dfeat (device M x in_dim, the features of the same states) is
 * needed in residual mode and may be NULL otherwise.                        */
MPPI_API int proposal_normalize(mppi_proposal p, const float* dU, const float* dfeat, int M,
                                float* dtarget);
/* One Adam step on the mean squared error of M rows (dfeat, dtarget device;
 * targets in scaled units).  loss_out (host, may be NULL) receives the loss
 * of the forward pass before the update (synchronous when given).          */
MPPI_API int proposal_train_step(mppi_proposal p, const float* dfeat, const float* dtarget, int M,
                                 float lr, float* loss_out);
/* Copy an intermediate of the last forward / training pass to the host (for
 * gradient checks): 0 pre-activation 1, 1 pre-activation 2, 2 output, 3 dOut,
 * 4 dH2, 5 dH1, 6 gradient vector (parameter layout); bf16 buffers widened to
 * float: 10 input, 11 activation 1, 12 activation 2, 13 dOut, 14 dH2, 15 dH1. */
MPPI_API int proposal_get_buffer(mppi_proposal p, int which, float* host, long long n);
/* Flat binary file: header, Adam step, scaling, parameters, Adam moments.   */
MPPI_API int proposal_save(mppi_proposal p, const char* path);
MPPI_API int proposal_load(mppi_proposal p, const char* path);

#ifdef __cplusplus
}
#endif

#endif /* EXACT_MPPI_H */
