// C ABI of the library (declared in include/exact_mppi.h): context, footprint
// and obstacle-set management, and the orchestration of one control cycle.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/exact_mppi.h"
#include "kernels.hpp"

#include "ctx.hpp"

using namespace emppi;
using namespace emppi_host;

static int rollout_into_ws(mppi_ctx ctx, const StepArgs& A, const float* dU, float* dposes,
                           float* deps, float* du, bool argmin, const float* useq = nullptr);

// Fixed device workspace of sdf_min_poses_noalloc: the merged distance keys
// of up to MPPI_NOALLOC_MAX_POSES poses (8 bytes each with the argmin, 4
// without).  Every device the library runs on holds its own copy for the
// life of the process.  In host code `scratch` names a host-side stand-in:
// kernels get the device address looked up per device by mppi_create.
static __device__ __align__(256) unsigned long long scratch[MPPI_NOALLOC_MAX_POSES];

namespace {

constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};

// Device address of `scratch` on the current device `device`, looked up once.
hipError_t scratch_lookup(int device) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_ptr[device] = p;
    return e;
}

void* scratch_ptr(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return device >= 0 && device < SCRATCH_MAX_DEVICES ? g_scratch_ptr[device] : nullptr;
}

}  // namespace

extern "C" {

int mppi_create(mppi_ctx* out, int device, void* hip_stream) {
    if (!out) return fail(nullptr, MPPI_E_ARG, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess) return fail(nullptr, MPPI_E_HIP, "hipGetDeviceCount: %s", hipGetErrorString(e));
    if (device < 0 || device >= n) return fail(nullptr, MPPI_E_ARG, "device %d of %d", device, n);
    mppi_ctx ctx = new mppi_ctx_s;
    ctx->device = device;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    DeviceGuard g(device);
    e = ctx->n_valid.ensure(sizeof(int));
    if (e == hipSuccess) e = ctx->path.ensure(MPPI_MAX_PATH * sizeof(float2));
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&ctx->h_out), OUT_FLOATS * sizeof(float), 0);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void**>(&ctx->h_res), OUT_FLOATS * sizeof(float),
                          hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess) e = hipHostGetDevicePointer(reinterpret_cast<void**>(&ctx->d_res), ctx->h_res, 0);
    if (e == hipSuccess) e = hipMemsetAsync(ctx->n_valid.p, 0, sizeof(int), ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e == hipSuccess) e = scratch_lookup(device);  // the device is current (DeviceGuard)
    if (e != hipSuccess) {
        mppi_destroy(ctx);
        return fail(nullptr, MPPI_E_HIP, "context setup: %s", hipGetErrorString(e));
    }
    *out = ctx;
    return MPPI_OK;
}

int mppi_destroy(mppi_ctx ctx) {
    if (!ctx) return MPPI_OK;
    {
        DeviceGuard g(ctx->device);
        (void)hipStreamSynchronize(ctx->stream);
        if (ctx->gbatch) mppi_batch_destroy(ctx->gbatch);
        DevBuf* bufs[] = {&ctx->poly_verts, &ctx->poly_tab_a, &ctx->poly_tab_b, &ctx->rects,
                          &ctx->px, &ctx->py, &ctx->pvx, &ctx->pvy, &ctx->pidx, &ctx->n_valid,
                          &ctx->path, &ctx->cloud_keys, &ctx->cloud_first, &ctx->cloud_cell,
                          &ctx->cloud_r2, &ctx->cloud_misc,
                          &ctx->eps_ws, &ctx->poses_ws, &ctx->jbase, &ctx->jt,
                          &ctx->key, &ctx->key64, &ctx->unew, &ctx->nom_poses,
                          &ctx->key_nom};
        for (DevBuf* b : bufs) b->release();
        if (ctx->h_out) (void)hipHostFree(ctx->h_out);
        if (ctx->h_res) (void)hipHostFree(ctx->h_res);
        if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
        if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    }
    delete ctx;
    return MPPI_OK;
}

const char* mppi_last_error(mppi_ctx ctx) {
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int mppi_check_footprint(int kind, const float* host, int count, char* msg, int msg_len) {
    mppi_ctx_s tmp;
    int rc = MPPI_OK;
    if (!host) {
        rc = fail(&tmp, MPPI_E_ARG, "footprint data is NULL");
    } else if (kind == MPPI_FP_POLYGON) {
        if (count < 3 || count > MPPI_MAX_B) {
            rc = fail(&tmp, MPPI_E_CAPACITY, "polygon needs 3..%d vertices, got %d", MPPI_MAX_B, count);
        } else {
            std::vector<double> v(2 * count);
            for (int k = 0; k < 2 * count; ++k) v[k] = host[k];
            rc = check_polygon(&tmp, v, count);
        }
    } else if (kind == MPPI_FP_RECTS) {
        if (count < 1 || count > MPPI_MAX_R) {
            rc = fail(&tmp, MPPI_E_CAPACITY, "rectangle cover needs 1..%d boxes, got %d", MPPI_MAX_R, count);
        } else {
            for (int j = 0; j < count && rc == MPPI_OK; ++j) {
                for (int k = 0; k < 4; ++k)
                    if (!std::isfinite(host[4 * j + k])) {
                        rc = fail(&tmp, MPPI_E_FOOTPRINT, "box %d not finite", j);
                        break;
                    }
                if (rc == MPPI_OK && (!(host[4 * j + 2] > 0) || !(host[4 * j + 3] > 0)))
                    rc = fail(&tmp, MPPI_E_FOOTPRINT, "box %d: half extents must be positive", j);
            }
        }
    } else {
        rc = fail(&tmp, MPPI_E_ARG, "unknown footprint kind %d", kind);
    }
    if (msg && msg_len > 0) {
        std::strncpy(msg, tmp.err.c_str(), static_cast<size_t>(msg_len) - 1);
        msg[msg_len - 1] = 0;
    }
    return rc;
}

int set_footprint(mppi_ctx ctx, int kind, const float* host, int count) {
    if (!ctx) return MPPI_E_ARG;
    {
        char msg[512];
        const int rc = mppi_check_footprint(kind, host, count, msg, sizeof msg);
        if (rc != MPPI_OK) return fail(ctx, rc, "%s", msg);
    }
    DeviceGuard g(ctx->device);
    if (kind == MPPI_FP_POLYGON) {
        const int BP = dmin_padded_count(0, count);
        // padded vertex list for the fused kernel: repeats of vertex 0
        std::vector<float> pv(2 * BP);
        for (int b = 0; b < BP; ++b) {
            const int s = b < count ? b : 0;
            pv[2 * b] = host[2 * s];
            pv[2 * b + 1] = host[2 * s + 1];
        }
        // point-wise tables, per edge taken from its lower end p towards its
        // upper end with unit direction e and length l: (ex, ey, -(e . p),
        // e x p) and (l, y of the edge's first vertex, 0, 0)
        std::vector<float> ta(4 * count), tb(4 * count);
        for (int b = 0; b < count; ++b) {
            const int n = (b + 1) % count;
            const double xa = host[2 * b], ya = host[2 * b + 1];
            const double xb = host[2 * n], yb = host[2 * n + 1];
            const bool down = yb < ya;
            const double px = down ? xb : xa, py = down ? yb : ya;
            const double dx = (down ? xa : xb) - px, dy = (down ? ya : yb) - py;
            const double l = std::sqrt(dx * dx + dy * dy);
            const double ex = l > 0.0 ? dx / l : 0.0, ey = l > 0.0 ? dy / l : 0.0;
            ta[4 * b] = static_cast<float>(ex);
            ta[4 * b + 1] = static_cast<float>(ey);
            ta[4 * b + 2] = static_cast<float>(-(ex * px + ey * py));
            ta[4 * b + 3] = l > 0.0 ? static_cast<float>(ey * px - ex * py) : 3.0e18f;
            tb[4 * b] = static_cast<float>(l);
            tb[4 * b + 1] = host[2 * b + 1];
            tb[4 * b + 2] = 0.0f;
            tb[4 * b + 3] = 0.0f;
        }
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        HIP_TRY(ctx, ctx->poly_verts.ensure(pv.size() * sizeof(float)));
        HIP_TRY(ctx, ctx->poly_tab_a.ensure(ta.size() * sizeof(float)));
        HIP_TRY(ctx, ctx->poly_tab_b.ensure(tb.size() * sizeof(float)));
        HIP_TRY(ctx, hipMemcpy(ctx->poly_verts.p, pv.data(), pv.size() * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(ctx, hipMemcpy(ctx->poly_tab_a.p, ta.data(), ta.size() * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(ctx, hipMemcpy(ctx->poly_tab_b.p, tb.data(), tb.size() * sizeof(float), hipMemcpyHostToDevice));
        ctx->B = count;
        ctx->BP = BP;
        ctx->has_poly = true;
        return MPPI_OK;
    }
    if (kind == MPPI_FP_RECTS) {
        const int RP = dmin_padded_count(1, count);
        std::vector<float> rv(4 * RP);
        for (int j = 0; j < RP; ++j)
            for (int k = 0; k < 4; ++k) rv[4 * j + k] = host[4 * (j < count ? j : 0) + k];
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        HIP_TRY(ctx, ctx->rects.ensure(rv.size() * sizeof(float)));
        HIP_TRY(ctx, hipMemcpy(ctx->rects.p, rv.data(), rv.size() * sizeof(float), hipMemcpyHostToDevice));
        ctx->R = count;
        ctx->RP = RP;
        ctx->has_rect = true;
        return MPPI_OK;
    }
    return fail(ctx, MPPI_E_ARG, "unknown footprint kind %d", kind);
}

int set_guidance(mppi_ctx ctx, const float* host_xy, int n) {
    if (!ctx) return MPPI_E_ARG;
    if (n < 0 || n > MPPI_MAX_PATH) return fail(ctx, MPPI_E_ARG, "guidance: n=%d outside [0, %d]", n, MPPI_MAX_PATH);
    if (n > 0 && !host_xy) return fail(ctx, MPPI_E_ARG, "guidance: NULL waypoints");
    for (int k = 0; k < 2 * n; ++k)
        if (!std::isfinite(host_xy[k])) return fail(ctx, MPPI_E_ARG, "guidance: non-finite waypoint");
    DeviceGuard g(ctx->device);
    if (n > 0) {
        HIP_TRY(ctx, hipMemcpyAsync(ctx->path.p, host_xy, sizeof(float2) * n, hipMemcpyHostToDevice,
                                    ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    }
    ctx->n_path = n;
    return MPPI_OK;
}

int set_points(mppi_ctx ctx, const float* dx, const float* dy, const float* dvx, const float* dvy,
               const unsigned char* dvalid, int n) {
    if (!ctx) return MPPI_E_ARG;
    if (n < 0) return fail(ctx, MPPI_E_ARG, "n < 0");
    if (n > 0 && (!dx || !dy)) return fail(ctx, MPPI_E_ARG, "point arrays are NULL");
    DeviceGuard g(ctx->device);
    const bool moving = dvx || dvy;
    const size_t cap = static_cast<size_t>(std::max(n, 1));
    HIP_TRY(ctx, ctx->px.ensure(cap * sizeof(float)));
    HIP_TRY(ctx, ctx->py.ensure(cap * sizeof(float)));
    HIP_TRY(ctx, ctx->pidx.ensure(cap * sizeof(int)));
    if (moving) {
        HIP_TRY(ctx, ctx->pvx.ensure(cap * sizeof(float)));
        HIP_TRY(ctx, ctx->pvy.ensure(cap * sizeof(float)));
        // a missing velocity component is zero
        if (!dvx) HIP_TRY(ctx, hipMemsetAsync(ctx->pvx.p, 0, cap * sizeof(float), ctx->stream));
        if (!dvy) HIP_TRY(ctx, hipMemsetAsync(ctx->pvy.p, 0, cap * sizeof(float), ctx->stream));
    }
    HIP_TRY(ctx, launch_compact_points(dx, dy, dvx, dvy, dvalid, n, ctx->px.as<float>(),
                                       ctx->py.as<float>(), dvx ? ctx->pvx.as<float>() : nullptr,
                                       dvy ? ctx->pvy.as<float>() : nullptr, ctx->pidx.as<int>(),
                                       ctx->n_valid.as<int>(), ctx->stream));
    ctx->n_points = n;
    ctx->moving = moving;
    return MPPI_OK;
}

int sdf_polygon(mppi_ctx ctx, const float* dpx, const float* dpy, int n, float* dd) {
    if (!ctx) return MPPI_E_ARG;
    if (n < 0 || (n > 0 && (!dpx || !dpy || !dd))) return fail(ctx, MPPI_E_ARG, "bad arrays");
    if (!ctx->has_poly) return fail(ctx, MPPI_E_NO_FOOTPRINT, "no polygon footprint set");
    DeviceGuard g(ctx->device);
    HIP_TRY(ctx, launch_sdf_points(0, dpx, dpy, n, ctx->poly_tab_a.as<float4>(),
                                   ctx->poly_tab_b.as<float4>(), ctx->B, dd, ctx->stream));
    return MPPI_OK;
}

int sdf_rectcover(mppi_ctx ctx, const float* dpx, const float* dpy, int n, float* dd) {
    if (!ctx) return MPPI_E_ARG;
    if (n < 0 || (n > 0 && (!dpx || !dpy || !dd))) return fail(ctx, MPPI_E_ARG, "bad arrays");
    if (!ctx->has_rect) return fail(ctx, MPPI_E_NO_FOOTPRINT, "no rectangle cover set");
    DeviceGuard g(ctx->device);
    HIP_TRY(ctx, launch_sdf_points(1, dpx, dpy, n, ctx->rects.as<float4>(), nullptr, ctx->R, dd,
                                   ctx->stream));
    return MPPI_OK;
}

int sdf_min_poses(mppi_ctx ctx, const float* dposes, int K, int T, float dt, int state_offset,
                  int kind, float* dd_min, int* dargmin) {
    if (!ctx) return MPPI_E_ARG;
    if (K < 0 || T < 1 || !dd_min || (K > 0 && !dposes)) return fail(ctx, MPPI_E_ARG, "bad arguments");
    if (kind == MPPI_FP_POLYGON && !ctx->has_poly) return fail(ctx, MPPI_E_NO_FOOTPRINT, "no polygon footprint set");
    if (kind == MPPI_FP_RECTS && !ctx->has_rect) return fail(ctx, MPPI_E_NO_FOOTPRINT, "no rectangle cover set");
    if (kind != MPPI_FP_POLYGON && kind != MPPI_FP_RECTS) return fail(ctx, MPPI_E_ARG, "kind %d", kind);
    const long long np = static_cast<long long>(K) * T;
    if (np > (1ll << 30)) return fail(ctx, MPPI_E_CAPACITY, "K*T too large");
    if (np == 0) return MPPI_OK;
    DeviceGuard g(ctx->device);
    PoseTime pt{1, T, state_offset ? 1 : 0, dt};
    unsigned int* key = nullptr;
    unsigned long long* key64 = nullptr;
    if (dargmin) {
        HIP_TRY(ctx, ctx->key64.ensure(sizeof(unsigned long long) * np));
        key64 = ctx->key64.as<unsigned long long>();
    } else {
        HIP_TRY(ctx, ctx->key.ensure(sizeof(unsigned int) * np));
        key = ctx->key.as<unsigned int>();
    }
    HIP_TRY(ctx, launch_key_init(key, key64, static_cast<int>(np), ctx->stream));
    if (int rc = run_dmin(ctx, reinterpret_cast<const float4*>(dposes), static_cast<int>(np), pt, kind,
                          key, key64))
        return rc;
    HIP_TRY(ctx, launch_dmin_finalize(key, key64, static_cast<int>(np), dd_min, dargmin, ctx->stream));
    return MPPI_OK;
}

int sdf_min_poses_noalloc(mppi_ctx ctx, const float* dposes, int K, int T, float dt,
                          int state_offset, int kind, float* dd_min, int* dargmin) {
    if (!ctx) return MPPI_E_ARG;
    if (K < 0 || T < 1 || (K > 0 && (!dposes || !dd_min))) return fail(ctx, MPPI_E_ARG, "bad arguments");
    if (kind == MPPI_FP_POLYGON && !ctx->has_poly) return fail(ctx, MPPI_E_NO_FOOTPRINT, "no polygon footprint set");
    if (kind == MPPI_FP_RECTS && !ctx->has_rect) return fail(ctx, MPPI_E_NO_FOOTPRINT, "no rectangle cover set");
    if (kind != MPPI_FP_POLYGON && kind != MPPI_FP_RECTS) return fail(ctx, MPPI_E_ARG, "kind %d", kind);
    const long long np = static_cast<long long>(K) * T;
    if (np > MPPI_NOALLOC_MAX_POSES)
        return fail(ctx, MPPI_E_CAPACITY, "K*T = %lld poses exceeds the fixed workspace of %d poses",
                    np, MPPI_NOALLOC_MAX_POSES);
    if (np == 0) return MPPI_OK;
    void* ws = scratch_ptr(ctx->device);
    if (!ws) return fail(ctx, MPPI_E_STATE, "fixed workspace not set up on device %d", ctx->device);
    DeviceGuard g(ctx->device);
    const PoseTime pt{1, T, state_offset ? 1 : 0, dt};
    unsigned int* key = dargmin ? nullptr : static_cast<unsigned int*>(ws);
    unsigned long long* key64 = dargmin ? static_cast<unsigned long long*>(ws) : nullptr;
    // the keys start at their +inf value (a kernel, no memset): the array
    // keeps whatever the previous call on this device left in it
    HIP_TRY(ctx, launch_key_init(key, key64, static_cast<int>(np), ctx->stream));
    if (int rc = run_dmin(ctx, reinterpret_cast<const float4*>(dposes), static_cast<int>(np), pt, kind,
                          key, key64))
        return rc;
    HIP_TRY(ctx, launch_dmin_finalize(key, key64, static_cast<int>(np), dd_min, dargmin, ctx->stream));
    return MPPI_OK;
}

static int rollout_into_ws(mppi_ctx ctx, const StepArgs& A, const float* dU, float* dposes,
                           float* deps, float* du, bool argmin, const float* useq) {
    const size_t Kpad = A.Kpad, T = A.T, nu = A.nu;
    HIP_TRY(ctx, ctx->eps_ws.ensure(sizeof(float) * T * nu * Kpad));
    HIP_TRY(ctx, ctx->poses_ws.ensure(sizeof(float4) * T * Kpad));
    HIP_TRY(ctx, ctx->jbase.ensure(sizeof(float) * Kpad));
    if (argmin)
        HIP_TRY(ctx, ctx->key64.ensure(sizeof(unsigned long long) * T * Kpad));
    else
        HIP_TRY(ctx, ctx->key.ensure(sizeof(unsigned int) * T * Kpad));
    RolloutOut o;
    o.eps_ws = ctx->eps_ws.as<float>();
    o.poses = ctx->poses_ws.as<float4>();
    o.jbase = ctx->jbase.as<float>();
    o.key = argmin ? nullptr : ctx->key.as<unsigned int>();
    o.key64 = argmin ? ctx->key64.as<unsigned long long>() : nullptr;
    o.diag_poses = dposes;
    o.diag_eps = deps;
    o.diag_u = du;
    o.useq = useq;
    HIP_TRY(ctx, launch_rollout(A, dU, o, ctx->stream));
    return MPPI_OK;
}

int mppi_sequence_costs(mppi_ctx ctx, const mppi_params* prm, const float* q0, const float* dUseq, int n,
                        float* dJ) {
    if (!ctx) return MPPI_E_ARG;
    if (!prm || !q0 || !dUseq || !dJ) return fail(ctx, MPPI_E_ARG, "NULL argument");
    if (n < 1 || n > MPPI_MAX_K) return fail(ctx, MPPI_E_CAPACITY, "n out of range");
    mppi_params p = *prm;
    p.K = n;
    if (int rc = check_params(ctx, &p)) return rc;
    DeviceGuard g(ctx->device);
    const StepArgs A = make_args(ctx, &p, q0, 0, 0);
    // rollouts of the given sequences (dU is not read in this mode)
    if (int rc = rollout_into_ws(ctx, A, dUseq, nullptr, nullptr, nullptr, false, dUseq)) return rc;
    const PoseTime pt{A.Kpad, A.T, A.state_offset, A.dt};
    if (int rc = run_dmin(ctx, ctx->poses_ws.as<float4>(), A.T * A.Kpad, pt, p.footprint_kind,
                          ctx->key.as<unsigned int>(), nullptr))
        return rc;
    HIP_TRY(ctx, ctx->jt.ensure(sizeof(float) * A.Kpad));
    HIP_TRY(ctx, launch_cost(A, ctx->key.as<unsigned int>(), nullptr, ctx->jbase.as<float>(),
                             ctx->jt.as<float>(), nullptr, nullptr, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(dJ, ctx->jt.p, sizeof(float) * n, hipMemcpyDeviceToDevice, ctx->stream));
    return MPPI_OK;
}

int mppi_rollout(mppi_ctx ctx, const mppi_params* prm, const float* q0, const float* dU,
                 uint64_t seed, uint64_t step, float* dposes, float* deps, float* du) {
    if (!ctx) return MPPI_E_ARG;
    if (!prm || !q0 || !dU) return fail(ctx, MPPI_E_ARG, "NULL argument");
    if (prm->K < 1 || prm->K > MPPI_MAX_K || prm->T < 1 || prm->T > MPPI_MAX_T)
        return fail(ctx, MPPI_E_CAPACITY, "K or T out of range");
    if (!valid_model(prm->model, prm->nu)) return fail(ctx, MPPI_E_ARG, "model/nu mismatch");
    DeviceGuard g(ctx->device);
    const StepArgs A = make_args(ctx, prm, q0, seed, step);
    return rollout_into_ws(ctx, A, dU, dposes, deps, du, false);
}

int mppi_set_graph(mppi_ctx ctx, int enable) {
    if (!ctx) return MPPI_E_ARG;
    ctx->graph_mode = enable != 0;
    if (!ctx->graph_mode && ctx->gbatch) {
        DeviceGuard g(ctx->device);
        mppi_batch_destroy(ctx->gbatch);
        ctx->gbatch = nullptr;
    }
    return MPPI_OK;
}

namespace {

// Graph-mode step: a one-scene batch of this context (bit-identical to the
// eager step) with an autotuned queue item size, rebuilt when the parameters
// change and re-planned when the points or the footprint changed.  With
// profiling on, the batch runs eagerly and its distance pass is timed.
int step_via_graph(mppi_ctx ctx, const mppi_params* prm, const float* q0, float* dU, uint64_t seed,
                   uint64_t step, float* u_out, int* valid_out) {
    if (ctx->gbatch && std::memcmp(&ctx->gprm, prm, sizeof(mppi_params)) != 0) {
        mppi_batch_destroy(ctx->gbatch);
        ctx->gbatch = nullptr;
    }
    // work the caller queued on the context's stream (nominal, points) comes first
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (!ctx->gbatch) {
        if (int rc = mppi_batch_create(&ctx->gbatch, &ctx, prm, 1, nullptr))
            return fail(ctx, rc, "graph mode: %s", mppi_batch_last_error(nullptr));
        ctx->gprm = *prm;
        if (int rc = mppi_batch_autotune(ctx->gbatch, 2, nullptr))
            return fail(ctx, rc, "graph mode: %s", mppi_batch_last_error(ctx->gbatch));
    }
    const int use_graph = ctx->prof ? 0 : 1;
    if (ctx->prof && mppi_batch_set_profiling(ctx->gbatch, 1) != MPPI_OK)
        return fail(ctx, MPPI_E_HIP, "graph mode: %s", mppi_batch_last_error(ctx->gbatch));
    int valid = 0;
    float u3[3];
    int rc = mppi_step_batched(ctx->gbatch, q0, dU, &seed, &step, u3, &valid, use_graph);
    if (rc == MPPI_E_STATE) {
        if ((rc = mppi_batch_refresh(ctx->gbatch)) == MPPI_OK)
            rc = mppi_step_batched(ctx->gbatch, q0, dU, &seed, &step, u3, &valid, use_graph);
    }
    if (rc) return fail(ctx, rc, "graph mode: %s", mppi_batch_last_error(ctx->gbatch));
    if (ctx->prof) {
        double ms = 0.0;
        long long n = 0;
        if ((rc = mppi_batch_get_profile(ctx->gbatch, &ms, &n)) != MPPI_OK ||
            (rc = mppi_batch_set_profiling(ctx->gbatch, 0)) != MPPI_OK)
            return fail(ctx, rc, "graph mode: %s", mppi_batch_last_error(ctx->gbatch));
        ctx->prof_ms += ms;
        ctx->prof_n += n;
    }
    for (int c = 0; c < prm->nu; ++c) u_out[c] = u3[c];
    if (valid_out) *valid_out = valid;
    return MPPI_OK;
}

}  // namespace

int mppi_step(mppi_ctx ctx, const mppi_params* prm, const float* q0, float* dU, uint64_t seed,
              uint64_t step, float* u_out, int* valid_out, const mppi_diag* diag) {
    if (!ctx) return MPPI_E_ARG;
    if (!q0 || !dU || !u_out) return fail(ctx, MPPI_E_ARG, "NULL argument");
    if (int rc = check_params(ctx, prm)) return rc;
    DeviceGuard g(ctx->device);
    if (ctx->graph_mode && !diag)
        return step_via_graph(ctx, prm, q0, dU, seed, step, u_out, valid_out);
    const StepArgs A = make_args(ctx, prm, q0, seed, step);
    const mppi_diag D = diag ? *diag : mppi_diag{};
    const int kind = prm->footprint_kind;
    const size_t Kpad = A.Kpad, T = A.T, nu = A.nu;

    // 1. sampling + rollouts (also initialises the distance keys)
    const bool argmin = D.argmin != nullptr;
    if (int rc = rollout_into_ws(ctx, A, dU, D.poses, D.eps, D.u, argmin)) return rc;
    unsigned int* key = argmin ? nullptr : ctx->key.as<unsigned int>();
    unsigned long long* key64 = argmin ? ctx->key64.as<unsigned long long>() : nullptr;
    // 2. signed distances, min over points
    PoseTime pt{A.Kpad, A.T, A.state_offset, A.dt};
    if (ctx->prof) HIP_TRY(ctx, hipEventRecord(ctx->ev0, ctx->stream));
    if (int rc = run_dmin(ctx, ctx->poses_ws.as<float4>(), static_cast<int>(T * Kpad), pt, kind, key,
                          key64))
        return rc;
    if (ctx->prof) HIP_TRY(ctx, hipEventRecord(ctx->ev1, ctx->stream));
    HIP_TRY(ctx, ctx->jt.ensure(sizeof(float) * Kpad));
    HIP_TRY(ctx, ctx->unew.ensure(sizeof(float) * T * nu));
    if (cost_update_fused(A.Kpad, A.T)) {
        // 2-3. costs, weights and update in one launch (small K)
        HIP_TRY(ctx, launch_cost_update(A, key, key64, ctx->jbase.as<float>(), ctx->eps_ws.as<float>(),
                                        dU, ctx->unew.as<float>(), ctx->jt.as<float>(), D.w, D.d_min,
                                        D.argmin, ctx->stream));
    } else {
        HIP_TRY(ctx, launch_cost(A, key, key64, ctx->jbase.as<float>(), ctx->jt.as<float>(), D.d_min,
                                 D.argmin, ctx->stream));
        // 3. weights and update
        HIP_TRY(ctx, launch_update(A, ctx->jt.as<float>(), ctx->eps_ws.as<float>(), dU,
                                   ctx->unew.as<float>(), D.w, ctx->stream));
    }
    if (D.J)
        HIP_TRY(ctx, hipMemcpyAsync(D.J, ctx->jt.p, sizeof(float) * A.K, hipMemcpyDeviceToDevice, ctx->stream));
    // 4. validation
    HIP_TRY(ctx, ctx->key_nom.ensure(sizeof(unsigned int) * T));
    const int padded = kind == MPPI_FP_POLYGON ? ctx->BP : ctx->RP;
    if (prm->validate && validate_small_supported(kind, padded) &&
        static_cast<long long>(T) * std::max(ctx->n_points, 0) * padded <= VAL_SMALL_MAX_PAIRS) {
        // nominal, its distances and validation in one single-workgroup launch
        HIP_TRY(ctx, launch_validate_small(A, kind, padded, point_args(ctx), ctx->poly_verts.as<float2>(),
                                           ctx->rects.as<float4>(), ctx->unew.as<float>(), dU,
                                           ctx->d_res, D.U_upd, D.d_nom, D.J_nom, ctx->stream));
    } else if (prm->validate) {
        HIP_TRY(ctx, ctx->nom_poses.ensure(sizeof(float4) * T));
        HIP_TRY(ctx, launch_nominal(A, ctx->unew.as<float>(), ctx->nom_poses.as<float4>(),
                                    ctx->key_nom.as<unsigned int>(), ctx->stream));
        PoseTime ptn{1, A.T, A.state_offset, A.dt};
        if (int rc = run_dmin(ctx, ctx->nom_poses.as<float4>(), A.T, ptn, kind,
                              ctx->key_nom.as<unsigned int>(), nullptr))
            return rc;
        HIP_TRY(ctx, launch_finalize(A, 1, ctx->key_nom.as<unsigned int>(), ctx->nom_poses.as<float4>(),
                                     ctx->unew.as<float>(), dU, ctx->d_res, D.U_upd, D.d_nom,
                                     D.J_nom, ctx->stream));
    } else {
        HIP_TRY(ctx, launch_finalize(A, 0, ctx->key_nom.as<unsigned int>(), ctx->nom_poses.as<float4>(),
                                     ctx->unew.as<float>(), dU, ctx->d_res, D.U_upd, D.d_nom,
                                     D.J_nom, ctx->stream));
    }
    // the finalising kernel wrote the result record into ctx->h_res
    // (device-mapped coherent host memory); the synchronisation makes it
    // visible here
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->prof) {
        float ms = 0.f;
        HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        ctx->prof_ms += ms;
        ctx->prof_n += 1;
    }
    for (int c = 0; c < prm->nu; ++c) u_out[c] = ctx->h_res[c];
    if (valid_out) *valid_out = ctx->h_res[3] != 0.0f;
    return MPPI_OK;
}

int mppi_autotune(mppi_ctx ctx, const mppi_params* prm, int reps, int* out_block, int* out_nchunk) {
    if (!ctx) return MPPI_E_ARG;
    if (int rc = check_params(ctx, prm)) return rc;
    if (reps < 1) reps = 3;
    DeviceGuard g(ctx->device);
    const float q0[3] = {0.f, 0.f, 0.f};
    const StepArgs A = make_args(ctx, prm, q0, 0x7E57ull, 0);
    // poses of one sampled step around a zero nominal
    HIP_TRY(ctx, ctx->unew.ensure(sizeof(float) * A.T * A.nu));
    HIP_TRY(ctx, hipMemsetAsync(ctx->unew.p, 0, sizeof(float) * A.T * A.nu, ctx->stream));
    if (int rc = rollout_into_ws(ctx, A, ctx->unew.as<float>(), nullptr, nullptr, nullptr, false)) return rc;
    const int kind = prm->footprint_kind;
    const int padded = kind == 0 ? ctx->BP : ctx->RP;
    const int npose = A.T * A.Kpad;
    PoseTime pt{A.Kpad, A.T, A.state_offset, A.dt};
    hipEvent_t e0, e1;
    HIP_TRY(ctx, hipEventCreate(&e0));
    HIP_TRY(ctx, hipEventCreate(&e1));
    const int blocks[] = {64, 128, 256};
    const int chunk_counts[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 13, 16, 20, 24, 32, 40, 48, 64, 96, 128};
    std::vector<std::pair<int, int>> cand;
    // chunks of at least 32 points, 8 when there are few poses (the pass then
    // needs the point chunks to fill the chip)
    const int min_chunk = npose <= 16384 ? 8 : 32;
    for (int b : blocks)
        for (int nc : chunk_counts)
            if (nc == 1 || ctx->n_points / nc >= min_chunk) cand.emplace_back(b, nc);
    std::vector<float> best(cand.size(), 1e30f);
    unsigned int* key = ctx->key.as<unsigned int>();
    int rc = MPPI_OK;
    // warm the clocks up first (about 40 launches of the default shape), then
    // time every candidate in a forward and a backward sweep and keep each
    // one's faster sweep, so clock ramps do not favour the later candidates
    for (int k = 0; k < 40 && rc == MPPI_OK; ++k)
        rc = run_dmin(ctx, ctx->poses_ws.as<float4>(), npose, pt, kind, key, nullptr);
    for (int sweep = 0; sweep < 2 && rc == MPPI_OK; ++sweep) {
        for (size_t n = 0; n < cand.size() && rc == MPPI_OK; ++n) {
            const size_t ci = sweep == 0 ? n : cand.size() - 1 - n;
            const int b = cand[ci].first, nc = cand[ci].second;
            // one untimed launch, then reps timed ones
            rc = run_dmin(ctx, ctx->poses_ws.as<float4>(), npose, pt, kind, key, nullptr, b, nc);
            if (rc) break;
            hipError_t e = hipEventRecord(e0, ctx->stream);
            for (int k = 0; k < reps && rc == MPPI_OK; ++k)
                rc = run_dmin(ctx, ctx->poses_ws.as<float4>(), npose, pt, kind, key, nullptr, b, nc);
            if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = fail(ctx, MPPI_E_HIP, "autotune timing: %s", hipGetErrorString(e));
                break;
            }
            best[ci] = std::min(best[ci], ms / reps);
        }
    }
    int best_b = 0, best_c = 0;
    float best_ms = 1e30f;
    for (size_t ci = 0; ci < cand.size(); ++ci)
        if (best[ci] < best_ms) {
            best_ms = best[ci];
            best_b = cand[ci].first;
            best_c = cand[ci].second;
        }
    if (rc == MPPI_OK)
        ctx->tuned[std::make_tuple(kind, padded, ctx->moving ? 1 : 0, npose, ctx->n_points)] = {best_b, best_c};
    // the validation pass (T poses of the nominal, one 64-lane workgroup per
    // point chunk): its chunk count, timed on the first T sampled poses
    if (rc == MPPI_OK && prm->validate) {
        const int nchunks[] = {8, 16, 32, 64, 128, 256, 512, 1024};
        std::vector<int> vc;
        for (int nc : nchunks)
            if (nc == 8 || ctx->n_points / nc >= 8) vc.push_back(nc);
        std::vector<float> vbest(vc.size(), 1e30f);
        const PoseTime ptn{1, A.T, A.state_offset, A.dt};
        HIP_TRY(ctx, ctx->key_nom.ensure(sizeof(unsigned int) * A.T));
        unsigned int* vkey = ctx->key_nom.as<unsigned int>();
        for (int sweep = 0; sweep < 2 && rc == MPPI_OK; ++sweep)
            for (size_t n = 0; n < vc.size() && rc == MPPI_OK; ++n) {
                const size_t ci = sweep == 0 ? n : vc.size() - 1 - n;
                rc = run_dmin(ctx, ctx->poses_ws.as<float4>(), A.T, ptn, kind, vkey, nullptr, 64, vc[ci]);
                if (rc) break;
                hipError_t e = hipEventRecord(e0, ctx->stream);
                for (int k = 0; k < reps && rc == MPPI_OK; ++k)
                    rc = run_dmin(ctx, ctx->poses_ws.as<float4>(), A.T, ptn, kind, vkey, nullptr, 64,
                                  vc[ci]);
                if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    rc = fail(ctx, MPPI_E_HIP, "autotune timing: %s", hipGetErrorString(e));
                    break;
                }
                vbest[ci] = std::min(vbest[ci], ms / reps);
            }
        if (rc == MPPI_OK) {
            size_t bi = 0;
            for (size_t ci = 1; ci < vc.size(); ++ci)
                if (vbest[ci] < vbest[bi]) bi = ci;
            ctx->tuned[std::make_tuple(kind, padded, ctx->moving ? 1 : 0, A.T, ctx->n_points)] = {64, vc[bi]};
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    if (out_block) *out_block = best_b;
    if (out_nchunk) *out_nchunk = best_c;
    return MPPI_OK;
}

int mppi_tune_get(mppi_ctx ctx, char* buf, int len) {
    if (!ctx || !buf || len < 1) return MPPI_E_ARG;
    std::string text;
    char line[160];
    for (const auto& kv : ctx->tuned) {
        std::snprintf(line, sizeof line, "%d %d %d %d %d %d %d\n", std::get<0>(kv.first),
                      std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
                      std::get<4>(kv.first), kv.second.first, kv.second.second);
        text += line;
    }
    if (static_cast<int>(text.size()) + 1 > len) return fail(ctx, MPPI_E_CAPACITY, "buffer too small");
    std::memcpy(buf, text.c_str(), text.size() + 1);
    return MPPI_OK;
}

int mppi_tune_set(mppi_ctx ctx, const char* text) {
    if (!ctx || !text) return MPPI_E_ARG;
    const char* p = text;
    while (*p) {
        int v[7];
        int used = 0;
        if (std::sscanf(p, "%d %d %d %d %d %d %d%n", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5], &v[6],
                        &used) != 7)
            break;
        if ((v[5] != 64 && v[5] != 128 && v[5] != 256) || v[6] < 1)
            return fail(ctx, MPPI_E_ARG, "bad tile line");
        ctx->tuned[std::make_tuple(v[0], v[1], v[2], v[3], v[4])] = {v[5], v[6]};
        p += used;
        while (*p == '\n' || *p == ' ' || *p == '\r') ++p;
    }
    return MPPI_OK;
}

int mppi_set_tiles(mppi_ctx ctx, int block, int nchunk) {
    if (!ctx) return MPPI_E_ARG;
    if (block != 0 && block != 64 && block != 128 && block != 256)
        return fail(ctx, MPPI_E_ARG, "block must be 0, 64, 128 or 256");
    if (block != 0 && nchunk < 1) return fail(ctx, MPPI_E_ARG, "nchunk must be >= 1");
    ctx->force_block = block;
    ctx->force_nchunk = block ? nchunk : 0;
    return MPPI_OK;
}

int mppi_set_profiling(mppi_ctx ctx, int enable) {
    if (!ctx) return MPPI_E_ARG;
    DeviceGuard g(ctx->device);
    if (enable && !ctx->ev0) {
        HIP_TRY(ctx, hipEventCreate(&ctx->ev0));
        HIP_TRY(ctx, hipEventCreate(&ctx->ev1));
    }
    ctx->prof = enable != 0;
    ctx->prof_ms = 0.0;
    ctx->prof_n = 0;
    return MPPI_OK;
}

int mppi_get_profile(mppi_ctx ctx, double* ms, long long* launches) {
    if (!ctx || !ms || !launches) return MPPI_E_ARG;
    *ms = ctx->prof_ms;
    *launches = ctx->prof_n;
    return MPPI_OK;
}

}  // extern "C"
