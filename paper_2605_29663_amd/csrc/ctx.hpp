// Host-side internals shared by the C ABI translation units: the context
// structure, device buffers, error reporting, argument checks and the
// launch planning of the fused signed-distance stage.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/exact_mppi.h"
#include "host_geom.hpp"
#include "kernels.hpp"

using emppi::DminLaunch;
using emppi::PointArgs;
using emppi::PoseTime;
using emppi::StepArgs;
using emppi::WAVE;

namespace emppi_host {

inline thread_local std::string g_create_error;

// A growable device buffer owned by the context.
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes) {
        if (bytes <= cap) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            cap = 0;
        }
        const size_t want = std::max<size_t>(bytes, 256);
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) cap = want;
        // EXACT_MPPI_POISON=1 fills every new workspace with 0xFF bytes (NaN
        // as float, the largest key as an integer), so that a kernel reading
        // a workspace entry no kernel wrote shows up in the results instead
        // of depending on what the allocator hands back
        if (e == hipSuccess && poison()) {
            e = hipMemset(p, 0xFF, want);
            if (e == hipSuccess) e = hipDeviceSynchronize();
        }
        return e;
    }
    static bool poison() {
        const char* v = std::getenv("EXACT_MPPI_POISON");
        return v && v[0] && v[0] != '0';
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        cap = 0;
    }
    template <typename T>
    T* as() const {
        return static_cast<T*>(p);
    }
};

}  // namespace emppi_host

using emppi_host::DevBuf;

struct mppi_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // footprint: polygon (padded vertices + point-wise tables) and rectangle cover
    bool has_poly = false, has_rect = false;
    int B = 0, BP = 0, R = 0, RP = 0;
    DevBuf poly_verts, poly_tab_a, poly_tab_b, rects;
    // obstacle points (compacted)
    int n_points = 0;
    bool moving = false;
    DevBuf px, py, pvx, pvy, pidx, n_valid;
    // guidance polyline (fixed capacity MPPI_MAX_PATH waypoints, so the
    // address a captured graph holds stays valid)
    DevBuf path;
    int n_path = 0;
    // point-cloud pre-processing workspace
    DevBuf cloud_keys, cloud_first, cloud_cell, cloud_r2, cloud_misc;
    // step workspaces
    DevBuf eps_ws, poses_ws, jbase, jt, key, key64, unew, nom_poses, key_nom;
    float* h_out = nullptr;  // pinned
    // the step's result record (u*, valid, J_nom), written by the last
    // kernel of a step straight into pinned, device-mapped, coherent host
    // memory (no device-to-host copy on the critical path): host address and
    // the device's address of the same memory
    float* h_res = nullptr;
    float* d_res = nullptr;
    // tile shapes picked by mppi_autotune, keyed by (kind, padded, moving, npose, n)
    std::map<std::tuple<int, int, int, int, int>, std::pair<int, int>> tuned;
    int force_block = 0, force_nchunk = 0;  // mppi_set_tiles
    // graph mode: steps without diagnostics replay a captured one-scene batch
    bool graph_mode = false;
    mppi_batch gbatch = nullptr;
    mppi_params gprm{};
    // profiling of the dominant launch
    bool prof = false;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    double prof_ms = 0.0;
    long long prof_n = 0;
};

namespace emppi_host {

inline int fail(mppi_ctx ctx, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_create_error = buf;
    return code;
}

#define HIP_TRY(ctx, expr)                                                                    \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess)                                                                 \
            return fail((ctx), MPPI_E_HIP, "%s failed: %s", #expr, hipGetErrorString(_e));    \
    } while (0)

// RAII guard that makes ctx->device current for the duration of a call.
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

// Simple-polygon check of set_footprint (host_geom.hpp holds the geometry).
inline int check_polygon(mppi_ctx ctx, const std::vector<double>& v, int B) {
    char msg[160];
    if (polygon_defect(v, B, msg, sizeof msg)) return fail(ctx, MPPI_E_FOOTPRINT, "%s", msg);
    return MPPI_OK;
}

inline bool valid_model(int model, int nu) {
    switch (model) {
    case MPPI_UNICYCLE:
    case MPPI_ACKERMANN: return nu == 2;
    case MPPI_OMNI: return nu == 3;
    case MPPI_SPIN:
    case MPPI_PARALLEL: return nu == 1;
    default: return false;
    }
}

inline int check_params(mppi_ctx ctx, const mppi_params* p) {
    if (!p) return fail(ctx, MPPI_E_ARG, "params is NULL");
    if (p->K < 1 || p->K > MPPI_MAX_K) return fail(ctx, MPPI_E_CAPACITY, "K=%d outside [1, %d]", p->K, MPPI_MAX_K);
    if (p->T < 1 || p->T > MPPI_MAX_T) return fail(ctx, MPPI_E_CAPACITY, "T=%d outside [1, %d]", p->T, MPPI_MAX_T);
    if (p->nu < 1 || p->nu > 3) return fail(ctx, MPPI_E_CAPACITY, "nu=%d outside [1, 3]", p->nu);
    if (!valid_model(p->model, p->nu)) return fail(ctx, MPPI_E_ARG, "model %d does not take nu=%d", p->model, p->nu);
    if (p->footprint_kind != MPPI_FP_POLYGON && p->footprint_kind != MPPI_FP_RECTS)
        return fail(ctx, MPPI_E_ARG, "footprint_kind %d", p->footprint_kind);
    if (!(p->dt > 0) || !(p->lambda > 0) || !std::isfinite(p->dt) || !std::isfinite(p->lambda))
        return fail(ctx, MPPI_E_ARG, "dt and lambda must be positive and finite");
    if (p->model == MPPI_ACKERMANN && !(p->wheelbase > 0))
        return fail(ctx, MPPI_E_ARG, "wheelbase must be positive");
    for (int c = 0; c < p->nu; ++c)
        if (!(p->u_min[c] <= p->u_max[c]) || !(p->sigma[c] >= 0))
            return fail(ctx, MPPI_E_ARG, "channel %d: need sigma >= 0 and u_min <= u_max", c);
    if (p->footprint_kind == MPPI_FP_POLYGON && !ctx->has_poly)
        return fail(ctx, MPPI_E_NO_FOOTPRINT, "no polygon footprint set");
    if (p->footprint_kind == MPPI_FP_RECTS && !ctx->has_rect)
        return fail(ctx, MPPI_E_NO_FOOTPRINT, "no rectangle cover set");
    return MPPI_OK;
}

inline StepArgs make_args(mppi_ctx ctx, const mppi_params* p, const float* q0, uint64_t seed,
                          uint64_t step) {
    StepArgs a{};
    a.path = ctx->path.as<float2>();
    a.n_path = ctx->n_path;
    a.w_path = p->w_path;
    a.K = p->K;
    a.Kpad = (p->K + WAVE - 1) / WAVE * WAVE;
    a.T = p->T;
    a.nu = p->nu;
    a.model = p->model;
    a.state_offset = p->state_offset ? 1 : 0;
    a.dt = p->dt;
    a.lambda = p->lambda;
    a.wheelbase = p->wheelbase;
    for (int c = 0; c < 3; ++c) {
        const bool on = c < p->nu;
        a.sigma[c] = on ? p->sigma[c] : 0.f;
        a.umin[c] = on ? p->u_min[c] : 0.f;
        a.umax[c] = on ? p->u_max[c] : 0.f;
        a.w_ctrl[c] = on ? p->w_ctrl[c] : 0.f;
        a.q0[c] = q0[c];
    }
    a.d_safe = p->d_safe;
    a.w_coll = p->w_coll;
    a.w_rep = p->w_rep;
    a.w_inf = p->w_inf;
    a.w_goal = p->w_goal;
    a.goal[0] = p->goal[0];
    a.goal[1] = p->goal[1];
    a.seed = seed;
    a.step = step;
    a.stream = 0;
    return a;
}

inline PointArgs point_args(mppi_ctx ctx) {
    PointArgs pa;
    pa.x = ctx->px.as<float>();
    pa.y = ctx->py.as<float>();
    pa.vx = ctx->moving ? ctx->pvx.as<float>() : nullptr;
    pa.vy = ctx->moving ? ctx->pvy.as<float>() : nullptr;
    pa.idx = ctx->pidx.as<int>();
    pa.n_valid = ctx->n_valid.as<int>();
    return pa;
}

// Waves per SIMD the fused kernel runs at (its register budget), used to
// estimate how many workgroups are resident at once.
inline int dmin_waves_per_simd(int kind, int padded) {
    if (kind == 1) return 8;
    // above 16 vertices a lane pair shares a pose (half the edges per lane),
    // above 32 a lane quad
    return padded <= 8 ? 6 : padded <= 16 ? 4 : 3;
}

// Default tile shape: chunks of at least 32 points, and a workgroup count
// close to a whole number of "rounds" of resident workgroups so that the
// last round is not a nearly empty tail (all workgroups do equal work).
inline void choose_tiles(int kind, int padded, int npose, int n_points, int& block, int& nchunk, int& chunk) {
    block = npose >= 4096 ? 256 : 64;
    const int lanes = kind == 0 && padded > 32 ? 4 : kind == 0 && padded > 16 ? 2 : 1;  // per pose
    const int pose_blocks = std::max(1, (lanes * npose + block - 1) / block);
    const int resident = 256 * 4 * dmin_waves_per_simd(kind, padded) / (block / WAVE);
    // a pass over few poses (the validation rollout) is bound by the serial
    // point loop of one wave: split the points finer
    const int max_chunks = std::max(1, n_points / (pose_blocks == 1 ? 16 : npose <= 16384 ? 8 : 32));
    int best_nc = 1;
    double best_eff = -1.0;
    for (int nc = 1; nc <= std::min(max_chunks, 4096); ++nc) {
        const long long wgs = static_cast<long long>(pose_blocks) * nc;
        const double rounds = static_cast<double>(wgs) / resident;
        const double eff = rounds / std::ceil(rounds);      // fill of the last round
        const double score = eff * std::min(1.0, rounds / 4.0);  // prefer >= 4 rounds
        if (score > best_eff + 1e-9) {
            best_eff = score;
            best_nc = nc;
        }
        if (rounds > 16) break;
    }
    chunk = std::max(1, (n_points + best_nc - 1) / best_nc);
    nchunk = std::max(1, (n_points + chunk - 1) / chunk);
}

// Launch shape of the fused transform + signed distance + min stage.
inline DminLaunch dmin_launch(mppi_ctx ctx, const float4* poses, int npose, PoseTime pt, int kind,
                              unsigned int* key, unsigned long long* key64, int force_block = 0,
                              int force_nchunk = 0) {
    const int padded = kind == 0 ? ctx->BP : ctx->RP;
    int block, nchunk, chunk;
    choose_tiles(kind, padded, npose, ctx->n_points, block, nchunk, chunk);
    const auto it = ctx->tuned.find(std::make_tuple(kind, padded, ctx->moving ? 1 : 0, npose, ctx->n_points));
    if (it != ctx->tuned.end()) {
        block = it->second.first;
        nchunk = it->second.second;
    }
    if (ctx->force_block) {
        block = ctx->force_block;
        nchunk = ctx->force_nchunk;
    }
    if (force_block) block = force_block;
    if (force_nchunk) nchunk = force_nchunk;
    chunk = std::max(1, (ctx->n_points + nchunk - 1) / nchunk);
    nchunk = std::max(1, (ctx->n_points + chunk - 1) / chunk);
    DminLaunch L{};
    L.poses = poses;
    L.npose = npose;
    L.pt = pt;
    L.pts = point_args(ctx);
    L.chunk = chunk;
    L.nchunk = nchunk;
    L.block = block;
    L.kind = kind;
    L.verts = ctx->poly_verts.as<float2>();
    L.rects = ctx->rects.as<float4>();
    L.padded = padded;
    L.argmin = key64 != nullptr;
    L.key = key;
    L.key64 = key64;
    return L;
}

// Fused transform + signed distance + min launch; the keys (key, or key64
// when argmin) must hold their initial values for the poses.
inline int run_dmin(mppi_ctx ctx, const float4* poses, int npose, PoseTime pt, int kind,
                    unsigned int* key, unsigned long long* key64, int force_block = 0,
                    int force_nchunk = 0) {
    const DminLaunch L = dmin_launch(ctx, poses, npose, pt, kind, key, key64, force_block, force_nchunk);
    HIP_TRY(ctx, launch_dmin(L, ctx->stream));
    return MPPI_OK;
}

}  // namespace emppi_host
