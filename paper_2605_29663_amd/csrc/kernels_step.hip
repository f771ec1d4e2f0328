// Single-scene kernels of the sampling + rollout, cost, path-integral update,
// nominal re-rollout and validation stages (Algorithm 1 steps 1, 2-3, 4).
// The per-workgroup work is in step_device.hpp (shared with the batched
// kernels).
#include "sdf_device.hpp"
#include "step_device.hpp"

namespace emppi {

namespace {

template <int RB, int HC>
__global__ __launch_bounds__(RB * HC) void k_rollout(StepArgs P, const float* __restrict__ U,
                                                     RolloutOut o) {
    __shared__ float lds[roll_lds_floats(RB, HC)];
    rollout_block<RB, HC>(P, U, o, blockIdx.x * RB, lds);
}

__global__ __launch_bounds__(COST_THREADS) void k_cost(StepArgs P,
                                                       const unsigned int* __restrict__ key,
                                                       const unsigned long long* __restrict__ key64,
                                                       const float* __restrict__ jbase,
                                                       float* __restrict__ jt,
                                                       float* __restrict__ diag_dmin,
                                                       int* __restrict__ diag_argmin) {
    __shared__ float lds[2 * COST_THREADS];
    cost_block(P, key, key64, jbase, jt, diag_dmin, diag_argmin, blockIdx.x * WAVE, lds);
}

__global__ __launch_bounds__(256) void k_update(StepArgs P, const float* __restrict__ jt,
                                                const float* __restrict__ eps_ws,
                                                const float* __restrict__ U,
                                                float* __restrict__ Unew,
                                                float* __restrict__ diag_w) {
    __shared__ float sh[16];
    update_block(P, jt, eps_ws, U, Unew, diag_w, blockIdx.x, sh);
}

__global__ __launch_bounds__(NOM_THREADS) void k_nominal(StepArgs P, const float* __restrict__ Unew,
                                                float4* __restrict__ nom,
                                                unsigned int* __restrict__ key_nom) {
    __shared__ float lds[NOM_LDS_FLOATS];
    nominal_block(P, Unew, nom, key_nom, lds);
}

__global__ __launch_bounds__(FIN_THREADS) void k_finalize(
    StepArgs P, int validate, const unsigned int* __restrict__ key_nom,
    const float4* __restrict__ nom, const float* __restrict__ Unew, float* __restrict__ U,
    float* __restrict__ out, float* __restrict__ diag_unew, float* __restrict__ diag_dnom,
    float* __restrict__ diag_jnom) {
    __shared__ float sh[16];
    finalize_block(P, validate, key_nom, nom, Unew, U, out, diag_unew, diag_dnom, diag_jnom, sh);
}

__global__ __launch_bounds__(COST_THREADS) void k_cost_update(StepArgs P,
                                                     const unsigned int* __restrict__ key,
                                                     const unsigned long long* __restrict__ key64,
                                                     const float* __restrict__ jbase,
                                                     const float* __restrict__ eps_ws,
                                                     const float* __restrict__ U,
                                                     float* __restrict__ Unew,
                                                     float* __restrict__ jt,
                                                     float* __restrict__ diag_w,
                                                     float* __restrict__ diag_dmin,
                                                     int* __restrict__ diag_argmin) {
    __shared__ float sP[(COST_THREADS / WAVE) * COST_UPDATE_MAX_KPAD];
    __shared__ unsigned char sC[(COST_THREADS / WAVE) * COST_UPDATE_MAX_KPAD];
    __shared__ float sJ[COST_UPDATE_MAX_KPAD];
    __shared__ float sh[16];
    cost_update_block(P, key, key64, jbase, eps_ws, U, Unew, jt, diag_w, diag_dmin, diag_argmin,
                      blockIdx.x, sP, sC, sJ, sh);
}

// Algorithm 1 step 4 in one workgroup for small T N: the nominal re-rollout
// (nominal_block), the signed distances of its T poses (every thread one
// pose and an interleaved subset of the points, the footprint rotated into
// the pose's frame as in the multi-workgroup pass, minima merged into LDS
// keys) and validation / shift / reset (finalize_block).  The nominal poses
// and keys never leave LDS; the results are those of the three separate
// launches bit for bit (the minima are exact, the rest is the same code).
template <int KIND, int PAD, bool MOVING>
__global__ __launch_bounds__(VAL_SMALL_THREADS) void k_validate_small(
    StepArgs P, PointArgs pts, const float2* __restrict__ verts, const float4* __restrict__ rects,
    const float* __restrict__ Unew, float* __restrict__ U, float* __restrict__ out,
    float* __restrict__ diag_unew, float* __restrict__ diag_dnom, float* __restrict__ diag_jnom) {
    __shared__ float lds_nom[NOM_LDS_FLOATS];
    __shared__ float4 nom[MPPI_MAX_T_DEV];
    __shared__ unsigned int skey[MPPI_MAX_T_DEV];
    __shared__ __align__(16) float tile[DMIN_TILE * (MOVING ? 4 : 2)];
    __shared__ float sh[16];
    // Loads that do not depend on the nominal are issued first, so that
    // their latency overlaps the nominal re-rollout: the valid count, the
    // first tile of points (one per thread: VAL_SMALL_THREADS == DMIN_TILE)
    // and the footprint.
    static_assert(VAL_SMALL_THREADS == DMIN_TILE, "one point of the first tile per thread");
    const int nv = *pts.n_valid;
    const int ti = static_cast<int>(threadIdx.x);
    float4 p0 = make_float4(0.f, 0.f, 0.f, 0.f);
    if (ti < nv) {
        p0.x = pts.x[ti];
        p0.y = pts.y[ti];
        if (MOVING) {
            p0.z = pts.vx[ti];
            p0.w = pts.vy[ti];
        }
    }
    // (polygons above 12 vertices read theirs after the nominal: held
    // through it, their vertices would push the frame's registers into
    // scratch)
    constexpr bool PRE_VERTS = KIND == 0 && PAD <= 12;
    float2 vtx[KIND == 0 ? PAD : 1];
    float4 bx[KIND == 1 ? PAD : 1];
    if constexpr (PRE_VERTS) {
#pragma unroll
        for (int k = 0; k < PAD; ++k) vtx[k] = verts[k];
    } else if constexpr (KIND == 1) {
#pragma unroll
        for (int k = 0; k < PAD; ++k) bx[k] = wave_uniform(rects[k]);
    }
    nominal_block(P, Unew, nom, skey, lds_nom);
    if (ti < min(nv, DMIN_TILE)) {
        if (MOVING)
            reinterpret_cast<float4*>(tile)[ti] = p0;
        else
            reinterpret_cast<float2*>(tile)[ti] = make_float2(p0.x, p0.y);
    }
    __syncthreads();
    const int T = P.T;
    const int S = static_cast<int>(blockDim.x) / T;  // point subsets per pose
    const int h = static_cast<int>(threadIdx.x) % T, j = static_cast<int>(threadIdx.x) / T;
    const bool act = j < S;
    const float4 q = nom[h];
    const PoseTime pt{1, T, P.state_offset, P.dt};
    const float tau = MOVING ? pose_tau(pt, h) : 0.0f;
    float best = INFINITY;
    int besti = -1;
    if constexpr (KIND == 0) {
        PolyFrame<PAD> F;
        if constexpr (PRE_VERTS)
            F.init_from(vtx, q.z, q.w);
        else
            F.init(verts, q.z, q.w);
        for (int t0 = 0; t0 < nv; t0 += DMIN_TILE) {
            const int tn = min(DMIN_TILE, nv - t0);
            if (t0 > 0) {
                __syncthreads();
                stage_points<MOVING>(tile, pts, t0, tn);
                __syncthreads();
            }
            if (act)
                for (int i = j; i < tn; i += S) {
                    float dx, dy;
                    point_rel<MOVING>(tile, i, tau, q.x, q.y, dx, dy);
                    take<false>(F.eval(dx, dy), t0 + i, best, besti);
                }
        }
    } else {
        for (int t0 = 0; t0 < nv; t0 += DMIN_TILE) {
            const int tn = min(DMIN_TILE, nv - t0);
            if (t0 > 0) {
                __syncthreads();
                stage_points<MOVING>(tile, pts, t0, tn);
                __syncthreads();
            }
            if (act)
                for (int i = j; i < tn; i += S) {
                    float dx, dy;
                    point_rel<MOVING>(tile, i, tau, q.x, q.y, dx, dy);
                    const float px = __builtin_fmaf(q.z, dx, q.w * dy);
                    const float py = __builtin_fmaf(q.z, dy, -(q.w * dx));
                    float sv = box_s(px, py, bx[0]);
#pragma unroll
                    for (int k = 1; k < PAD; ++k) sv = fminf(sv, box_s(px, py, bx[k]));
                    take<false>(sv, t0 + i, best, besti);
                }
        }
    }
    if (act) atomicMin(&skey[h], dkey(best));
    __syncthreads();
    finalize_block(P, 1, skey, nom, Unew, U, out, diag_unew, diag_dnom, diag_jnom, sh);
}

template <int KIND, int PAD>
hipError_t launch_validate_small_t(const StepArgs& P, const PointArgs& pts, const float2* verts,
                                   const float4* rects, const float* Unew, float* U, float* out,
                                   float* diag_unew, float* diag_dnom, float* diag_jnom,
                                   hipStream_t s) {
    if (pts.vx)
        hipLaunchKernelGGL((k_validate_small<KIND, PAD, true>), dim3(1), dim3(VAL_SMALL_THREADS), 0, s,
                           P, pts, verts, rects, Unew, U, out, diag_unew, diag_dnom, diag_jnom);
    else
        hipLaunchKernelGGL((k_validate_small<KIND, PAD, false>), dim3(1), dim3(VAL_SMALL_THREADS), 0,
                           s, P, pts, verts, rects, Unew, U, out, diag_unew, diag_dnom, diag_jnom);
    return hipGetLastError();
}

}  // namespace

bool validate_small_supported(int kind, int padded) {
    return kind == 1 ? padded <= 12 : padded >= 3 && padded <= 16;
}

hipError_t launch_validate_small(const StepArgs& P, int kind, int padded, const PointArgs& pts,
                                 const float2* verts, const float4* rects, const float* Unew,
                                 float* U, float* out, float* diag_unew, float* diag_dnom,
                                 float* diag_jnom, hipStream_t s) {
#define EMPPI_VS(KD, PD)                                                                       \
    case PD:                                                                                   \
        return launch_validate_small_t<KD, PD>(P, pts, verts, rects, Unew, U, out, diag_unew,  \
                                               diag_dnom, diag_jnom, s);
    if (kind == 0) {
        switch (padded) {
            EMPPI_VS(0, 3) EMPPI_VS(0, 4) EMPPI_VS(0, 5) EMPPI_VS(0, 6) EMPPI_VS(0, 7)
            EMPPI_VS(0, 8) EMPPI_VS(0, 9) EMPPI_VS(0, 10) EMPPI_VS(0, 11) EMPPI_VS(0, 12)
            EMPPI_VS(0, 13) EMPPI_VS(0, 14) EMPPI_VS(0, 15) EMPPI_VS(0, 16)
        default: return hipErrorInvalidValue;
        }
    }
    switch (padded) {
        EMPPI_VS(1, 1) EMPPI_VS(1, 2) EMPPI_VS(1, 3) EMPPI_VS(1, 4) EMPPI_VS(1, 6)
        EMPPI_VS(1, 8) EMPPI_VS(1, 12)
    default: return hipErrorInvalidValue;
    }
#undef EMPPI_VS
}

hipError_t launch_cost_update(const StepArgs& P, const unsigned int* key,
                              const unsigned long long* key64, const float* jbase,
                              const float* eps_ws, const float* U, float* Unew, float* jt,
                              float* diag_w, float* diag_dmin, int* diag_argmin, hipStream_t s) {
    if (!cost_update_fused(P.Kpad, P.T)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cost_update, dim3(P.T), dim3(COST_THREADS), 0, s, P, key, key64, jbase,
                       eps_ws, U, Unew, jt, diag_w, diag_dmin, diag_argmin);
    return hipGetLastError();
}

hipError_t launch_rollout(const StepArgs& P, const float* U, const RolloutOut& o, hipStream_t s) {
    // up to 2^14 rollouts: 16-rollout workgroups (more compute units on the
    // serial recursions), with the whole horizon in one chunk of 32 steps
    // when it fits (one noise pass and one pass of each recursion instead of
    // two); above, 64-rollout workgroups
    if (P.Kpad <= (1 << 14) && P.T > ROLL_HCHUNK && P.T <= 2 * ROLL_HCHUNK)
        hipLaunchKernelGGL((k_rollout<ROLL_RB_SMALL, 2 * ROLL_HCHUNK>), dim3(P.Kpad / ROLL_RB_SMALL),
                           dim3(ROLL_RB_SMALL * 2 * ROLL_HCHUNK), 0, s, P, U, o);
    else if (P.Kpad <= (1 << 14))
        hipLaunchKernelGGL((k_rollout<ROLL_RB_SMALL, ROLL_HCHUNK>), dim3(P.Kpad / ROLL_RB_SMALL),
                           dim3(ROLL_RB_SMALL * ROLL_HCHUNK), 0, s, P, U, o);
    else
        hipLaunchKernelGGL((k_rollout<WAVE, ROLL_HCHUNK>), dim3(P.Kpad / WAVE), dim3(ROLL_THREADS), 0, s,
                           P, U, o);
    return hipGetLastError();
}

hipError_t launch_cost(const StepArgs& P, const unsigned int* key, const unsigned long long* key64,
                       const float* jbase, float* jt, float* diag_dmin, int* diag_argmin,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_cost, dim3(P.Kpad / WAVE), dim3(COST_THREADS), 0, s, P, key, key64, jbase,
                       jt, diag_dmin, diag_argmin);
    return hipGetLastError();
}

hipError_t launch_update(const StepArgs& P, const float* jt, const float* eps_ws, const float* U,
                         float* Unew, float* diag_w, hipStream_t s) {
    hipLaunchKernelGGL(k_update, dim3(P.T), dim3(256), 0, s, P, jt, eps_ws, U, Unew, diag_w);
    return hipGetLastError();
}

hipError_t launch_nominal(const StepArgs& P, const float* Unew, float4* nom, unsigned int* key_nom,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_nominal, dim3(1), dim3(NOM_THREADS), 0, s, P, Unew, nom, key_nom);
    return hipGetLastError();
}

hipError_t launch_finalize(const StepArgs& P, int validate, const unsigned int* key_nom,
                           const float4* nom, const float* Unew, float* U, float* out,
                           float* diag_unew, float* diag_dnom, float* diag_jnom, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(FIN_THREADS), 0, s, P, validate, key_nom, nom, Unew,
                       U, out, diag_unew, diag_dnom, diag_jnom);
    return hipGetLastError();
}

}  // namespace emppi
