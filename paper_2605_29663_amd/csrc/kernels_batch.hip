// Batched kernels: one control cycle of many independent scenes of uneven
// size (rollouts, horizon, points, footprint) with a fixed number of launches.
// Every workgroup runs the same device functions as the single-scene kernels
// on its scene's arguments, so each scene's results are bit-identical to a
// single-scene step with the same inputs.
//
// The signed-distance stage is one persistent kernel per register class:
// workgroups pull (scene, pose tile, point chunk) items from a queue ordered
// longest-first, so scenes of very different cost share the chip without a
// tail of idle compute units.
#include "sdf_device.hpp"
#include "step_device.hpp"

namespace emppi {

namespace {

__global__ void k_batch_reset(int* counters, int n) {
    if (threadIdx.x < n) counters[threadIdx.x] = 0;
}

__global__ __launch_bounds__(ROLL_THREADS) void k_rollout_b(const SceneStep* __restrict__ steps,
                                                   const SceneBufs* __restrict__ bufs,
                                                   const int2* __restrict__ blk) {
    __shared__ float lds[ROLL_LDS_FLOATS];
    const int2 b = blk[blockIdx.x];  // (scene, first rollout)
    const SceneStep& S = steps[b.x];
    const SceneBufs& B = bufs[b.x];
    RolloutOut o;
    o.eps_ws = B.eps_ws;
    o.poses = B.poses;
    o.jbase = B.jbase;
    o.key = B.key;
    o.key64 = nullptr;
    o.diag_poses = nullptr;
    o.diag_eps = nullptr;
    o.diag_u = nullptr;
    rollout_block(S.P, S.U, o, b.y, lds);
}

// Footprint bucket dispatch over the register classes of dmin_class.
template <int CLS>
__device__ __forceinline__ void dmin_dispatch(const SceneDmin& S, bool moving, float4 q, float tau,
                                              int c0, int c1, float* lds, float& best) {
    int bi;
#define EMPPI_POLY(P)                                                                         \
    case P:                                                                                   \
        if (moving)                                                                           \
            dmin_poly_range<P, true, false>(q, tau, S.pts, c0, c1, S.verts, lds, best, bi);   \
        else                                                                                  \
            dmin_poly_range<P, false, false>(q, tau, S.pts, c0, c1, S.verts, lds, best, bi);  \
        return;
#define EMPPI_PART(P, L)                                                                      \
    case P:                                                                                   \
        if (moving)                                                                           \
            dmin_poly_part_range<P / L, L, true>(q, tau, S.pts, c0, c1, S.verts, lds, best, bi);  \
        else                                                                                  \
            dmin_poly_part_range<P / L, L, false>(q, tau, S.pts, c0, c1, S.verts, lds, best, bi); \
        return;
#define EMPPI_RECT(P)                                                                         \
    case P:                                                                                   \
        if (moving)                                                                           \
            dmin_rect_range<P, true, false>(q, tau, S.pts, c0, c1, S.rects, lds, best, bi);   \
        else                                                                                  \
            dmin_rect_range<P, false, false>(q, tau, S.pts, c0, c1, S.rects, lds, best, bi);  \
        return;
    if (CLS == 0) {
        switch (S.padded) {
            EMPPI_POLY(3)
            EMPPI_POLY(4)
            EMPPI_POLY(5)
            EMPPI_POLY(6)
            EMPPI_POLY(7)
            EMPPI_POLY(8)
        default: break;
        }
    } else if (CLS == 1) {
        switch (S.padded) {
            EMPPI_POLY(9)
            EMPPI_POLY(10)
            EMPPI_POLY(11)
            EMPPI_POLY(12)
            EMPPI_POLY(13)
            EMPPI_POLY(14)
            EMPPI_POLY(15)
            EMPPI_POLY(16)
        default: break;
        }
    } else if (CLS == 2) {
        switch (S.padded) {
            EMPPI_PART(18, 2)
            EMPPI_PART(20, 2)
            EMPPI_PART(22, 2)
            EMPPI_PART(24, 2)
            EMPPI_PART(26, 2)
            EMPPI_PART(28, 2)
            EMPPI_PART(30, 2)
        default: break;
        }
    } else if (CLS == 3) {
        switch (S.padded) {
            EMPPI_PART(32, 2)
        default: break;
        }
    } else if (CLS == 6) {
        switch (S.padded) {
            EMPPI_PART(36, 4)
            EMPPI_PART(40, 4)
            EMPPI_PART(44, 4)
            EMPPI_PART(48, 4)
            EMPPI_PART(52, 4)
            EMPPI_PART(56, 4)
            EMPPI_PART(60, 4)
            EMPPI_PART(64, 4)
        default: break;
        }
    } else if (CLS == 4) {
        switch (S.padded) {
            EMPPI_RECT(1)
            EMPPI_RECT(2)
            EMPPI_RECT(3)
            EMPPI_RECT(4)
            EMPPI_RECT(6)
            EMPPI_RECT(8)
            EMPPI_RECT(12)
        default: break;
        }
    } else if (CLS == 5) {
        switch (S.padded) {
            EMPPI_RECT(16)
            EMPPI_RECT(24)
            EMPPI_RECT(32)
        default: break;
        }
    }
#undef EMPPI_POLY
#undef EMPPI_PART
#undef EMPPI_RECT
    best = INFINITY;  // unreachable for planned items
}

// Waves per SIMD each register class is compiled for (its register budget).
template <int CLS>
constexpr int persistent_waves() {
    constexpr int waves[DMIN_CLASSES] = {6, 4, 4, 3, 8, 2, 3};
    return waves[CLS];
}

template <int CLS>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(persistent_waves<CLS>())))
void k_dmin_persistent(const SceneDmin* __restrict__ sds, const DminItem* __restrict__ items,
                       int n_items, int* __restrict__ counter) {
    extern __shared__ __align__(16) float lds[];  // point tiles: 8- and 16-byte LDS accesses
    __shared__ int next;
    for (;;) {
        __syncthreads();  // the previous item's LDS tile and `next` are no longer read
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        // the item is the same for the whole workgroup: keep it (and all
        // that is read through it) in scalar registers
        const int it = __builtin_amdgcn_readfirstlane(next);
        if (it >= n_items) break;
        const DminItem w = wave_uniform(items[it]);
        const SceneDmin S = wave_uniform(sds[w.sd]);
        // lane-group classes: dmin_class_lanes(CLS) lanes per pose
        constexpr int L = dmin_class_lanes(CLS);
        const int g = w.g0 + static_cast<int>(threadIdx.x / L);
        const int npose = S.npose;
        const bool live = g < npose;
        const float4 q = live ? S.poses[g] : make_float4(0.f, 0.f, 1.f, 0.f);
        const bool moving = S.pts.vx != nullptr;
        const float tau = moving ? pose_tau(S.pt, g) : 0.0f;
        const int nv = __builtin_amdgcn_readfirstlane(*S.pts.n_valid);
        const int c0 = w.c0;
        const int c1 = min(w.c1, nv);
        float best;
        dmin_dispatch<CLS>(S, moving, q, tau, c0, c1, lds, best);
        if (live && (threadIdx.x & (L - 1)) == 0) atomicMin(&S.key[g], dkey(best));
    }
}

__global__ __launch_bounds__(COST_THREADS) void k_cost_b(const SceneStep* __restrict__ steps,
                                                         const SceneBufs* __restrict__ bufs,
                                                         const int2* __restrict__ blk) {
    __shared__ float lds[2 * COST_THREADS];
    const int2 b = blk[blockIdx.x];
    const SceneBufs& B = bufs[b.x];
    cost_block(steps[b.x].P, B.key, nullptr, B.jbase, B.jt, nullptr, nullptr, b.y, lds);
}

__global__ __launch_bounds__(256) void k_update_b(const SceneStep* __restrict__ steps,
                                                  const SceneBufs* __restrict__ bufs,
                                                  const int2* __restrict__ blk) {
    __shared__ float sh[16];
    const int2 b = blk[blockIdx.x];  // (scene, horizon step)
    const SceneStep& S = steps[b.x];
    const SceneBufs& B = bufs[b.x];
    update_block(S.P, B.jt, B.eps_ws, S.U, B.unew, nullptr, b.y, sh);
}

__global__ __launch_bounds__(NOM_THREADS) void k_nominal_b(const SceneStep* __restrict__ steps,
                                                  const SceneBufs* __restrict__ bufs) {
    __shared__ float lds[NOM_LDS_FLOATS];
    const SceneBufs& B = bufs[blockIdx.x];
    nominal_block(steps[blockIdx.x].P, B.unew, B.nom, B.key_nom, lds);
}

__global__ __launch_bounds__(FIN_THREADS) void k_finalize_b(const SceneStep* __restrict__ steps,
                                                            const SceneBufs* __restrict__ bufs) {
    const SceneStep& S = steps[blockIdx.x];
    const SceneBufs& B = bufs[blockIdx.x];
    __shared__ float sh[16];
    finalize_block(S.P, B.validate, B.key_nom, B.nom, B.unew, S.U, B.out, nullptr, nullptr, nullptr,
                   sh);
}

// Diagnostics of one scene from its workspace: thread g < K*T handles pose
// (r, h) = (g / T, g % T); the first K, T*nu and T threads also copy J~, the
// updated nominal and the validation distances.
__global__ void k_scene_diag(SceneBufs B, int K, int Kpad, int T, int nu, SceneDiag d) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < K * T) {
        const int r = g / T, h = g - r * T;
        const int src = h * Kpad + r;
        if (d.d_min) d.d_min[g] = dkey_distance(B.key[src]);
        if (d.poses) {
            const float4 q = B.poses[src];
            d.poses[4 * static_cast<size_t>(g)] = q.x;
            d.poses[4 * static_cast<size_t>(g) + 1] = q.y;
            d.poses[4 * static_cast<size_t>(g) + 2] = q.z;
            d.poses[4 * static_cast<size_t>(g) + 3] = q.w;
        }
        if (d.eps)
            for (int c = 0; c < nu; ++c)
                d.eps[static_cast<size_t>(g) * nu + c] = B.eps_ws[(h * nu + c) * Kpad + r];
    }
    if (d.J && g < K) d.J[g] = B.jt[g];
    if (d.U_upd && g < T * nu) d.U_upd[g] = B.unew[g];
    if (d.d_nom && g < T) d.d_nom[g] = B.validate ? dkey_distance(B.key_nom[g]) : NAN;
    if (d.J_nom && g == 0) d.J_nom[0] = B.out[4];
}

// Hybrid-mode selection (Algorithm 2 steps 2-3), one thread: penalised costs
// Jbar_m = J_m + lambda_switch [m != m_prev] for validated modes (else
// +inf); safe stop (zero command, previous mode) when no mode validated;
// otherwise the lowest-index argmin, held at m_prev while the cooldown runs;
// then the command of the chosen mode with the velocity / yaw-rate deadzone
// correction.  `out` holds each mode's result record (OUT_FLOATS floats).
__global__ void k_hybrid_select(const float* __restrict__ out, HybridArgs a, float* __restrict__ res) {
    if (threadIdx.x != 0) return;
    float best = INFINITY;
    int mstar = -1;
    for (int m = 0; m < a.n_modes; ++m) {
        const float* o = out + m * OUT_FLOATS;
        const float jb = o[3] != 0.0f ? o[4] + (m != a.m_prev ? a.lambda_switch : 0.0f) : INFINITY;
        if (jb < best) {
            best = jb;
            mstar = m;
        }
    }
    for (int k = 0; k < OUT_FLOATS; ++k) res[k] = 0.0f;
    if (mstar < 0) {  // every mode failed validation
        res[3] = static_cast<float>(a.m_prev);
        res[4] = static_cast<float>(a.tau_cool);
        res[5] = 1.0f;
        res[6] = INFINITY;
        return;
    }
    if (a.tau_cool > 0 && mstar != a.m_prev) mstar = a.m_prev;
    const int tau = mstar != a.m_prev ? a.cool_max : max(a.tau_cool - 1, 0);
    const float* o = out + mstar * OUT_FLOATS;
    const int model = a.model[mstar], nu = a.nu[mstar];
    float u[3];
    for (int k = 0; k < 3; ++k) u[k] = k < nu ? o[k] : 0.0f;  // command structure of mode m*
    if (model != 3) {
        // translational modes: linear part (v) or (vx, vy) for the omni model
        const int nlin = model == 2 ? 2 : 1;
        float v2 = 0.0f;
        for (int k = 0; k < nlin; ++k) v2 += u[k] * u[k];
        const float vmag = __builtin_sqrtf(v2);
        if (a.noise_v < vmag && vmag < a.v_min) {
            const float sc = a.v_min / vmag;
            for (int k = 0; k < nlin; ++k) u[k] *= sc;
        }
    } else {
        // spin in place: yaw rate
        const float w = u[0];
        if (a.noise_w < fabsf(w) && fabsf(w) < a.w_min) u[0] = copysignf(a.w_min, w);
    }
    for (int k = 0; k < 3; ++k) res[k] = u[k];
    res[3] = static_cast<float>(mstar);
    res[4] = static_cast<float>(tau);
    res[5] = 0.0f;
    const float* os = out + mstar * OUT_FLOATS;
    res[6] = os[3] != 0.0f ? os[4] + (mstar != a.m_prev ? a.lambda_switch : 0.0f) : INFINITY;
}

}  // namespace

hipError_t launch_hybrid_select(const float* out, const HybridArgs& a, float* res, hipStream_t s) {
    hipLaunchKernelGGL(k_hybrid_select, dim3(1), dim3(64), 0, s, out, a, res);
    return hipGetLastError();
}

// LDS tile of the persistent kernels, sized for moving points (16 bytes per point)
constexpr size_t PERSISTENT_LDS = static_cast<size_t>(DMIN_TILE) * 16;

using PersistentKernel = void (*)(const SceneDmin*, const DminItem*, int, int*);
constexpr PersistentKernel PERSISTENT[DMIN_CLASSES] = {
    k_dmin_persistent<0>, k_dmin_persistent<1>, k_dmin_persistent<2>, k_dmin_persistent<3>,
    k_dmin_persistent<4>, k_dmin_persistent<5>, k_dmin_persistent<6>};

int dmin_persistent_blocks_per_cu(int cls, int block) {
    if (cls < 0 || cls >= DMIN_CLASSES) return 0;
    int nb = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &nb, reinterpret_cast<const void*>(PERSISTENT[cls]), block, PERSISTENT_LDS);
    return e == hipSuccess ? nb : 0;
}
int dmin_persistent_lanes_per_pose(int cls) { return dmin_class_lanes(cls); }

hipError_t launch_batch_reset(int* counters, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, counters, n);
    return hipGetLastError();
}

hipError_t launch_rollout_batched(const SceneStep* steps, const SceneBufs* bufs, const int2* blk,
                                  int nblk, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rollout_b, dim3(nblk), dim3(ROLL_THREADS), 0, s, steps, bufs, blk);
    return hipGetLastError();
}

hipError_t launch_dmin_persistent(int cls, int block, int grid, const SceneDmin* sds,
                                  const DminItem* items, int n_items, int* counter, hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (cls < 0 || cls >= DMIN_CLASSES) return hipErrorInvalidValue;
    hipLaunchKernelGGL(PERSISTENT[cls], dim3(grid), dim3(block), PERSISTENT_LDS, s, sds, items,
                       n_items, counter);
    return hipGetLastError();
}

hipError_t launch_cost_batched(const SceneStep* steps, const SceneBufs* bufs, const int2* blk,
                               int nblk, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cost_b, dim3(nblk), dim3(COST_THREADS), 0, s, steps, bufs, blk);
    return hipGetLastError();
}

hipError_t launch_update_batched(const SceneStep* steps, const SceneBufs* bufs, const int2* blk,
                                 int nblk, hipStream_t s) {
    if (nblk <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_update_b, dim3(nblk), dim3(256), 0, s, steps, bufs, blk);
    return hipGetLastError();
}

hipError_t launch_nominal_batched(const SceneStep* steps, const SceneBufs* bufs, int n,
                                  hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nominal_b, dim3(n), dim3(NOM_THREADS), 0, s, steps, bufs);
    return hipGetLastError();
}

hipError_t launch_scene_diag(const SceneBufs& B, int K, int Kpad, int T, int nu,
                             const SceneDiag& d, hipStream_t s) {
    const long long n = std::max(static_cast<long long>(K) * T, 3ll * T);
    const int blocks = static_cast<int>((n + 255) / 256);
    hipLaunchKernelGGL(k_scene_diag, dim3(blocks), dim3(256), 0, s, B, K, Kpad, T, nu, d);
    return hipGetLastError();
}

hipError_t launch_finalize_batched(const SceneStep* steps, const SceneBufs* bufs, int n,
                                   hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finalize_b, dim3(n), dim3(FIN_THREADS), 0, s, steps, bufs);
    return hipGetLastError();
}

}  // namespace emppi
