// Internal interface between the C ABI layer and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace emppi {

constexpr int WAVE = 64;
constexpr int DMIN_TILE = 1024;      // points staged in LDS per tile
constexpr int MPPI_MAX_T_DEV = 128;  // horizon capacity (MPPI_MAX_T of the C ABI)
// Per-step result record: u*_0, u*_1, u*_2, valid, J_nom (noise-free cost of
// the validated nominal), then padding.
constexpr int OUT_FLOATS = 8;

// Step parameters as the kernels see them (POD, passed by value).
struct StepArgs {
    int K, Kpad, T, nu, model, state_offset;
    float dt, lambda, wheelbase;
    float sigma[3], umin[3], umax[3];
    float d_safe, w_coll, w_rep, w_inf, w_goal, w_ctrl[3], goal[2];
    float q0[3];
    uint64_t seed, step, stream;
    const float2* path;  // guidance waypoints (planning frame)
    int n_path;
    float w_path;
};

// Valid obstacle points, compacted in index order (the count lives on the
// device so that a mask change needs no host round trip).
struct PointArgs {
    const float* x;
    const float* y;
    const float* vx;  // nullptr for static point sets
    const float* vy;
    const int* idx;   // caller's index of each compacted point
    const int* n_valid;
};

// Time of pose g for moving points: h = (g / div) % mod, t = (h + off) dt.
struct PoseTime {
    int div, mod, off;
    float dt;
};

// Order-preserving keys of the signed squared distance s: the unsigned order
// of key(s) is the order of s (sign bit flipped for s >= 0, all bits for
// s < 0).  Chunks of points merge their minima with atomicMin on these keys
// (exact and order-independent, hence deterministic); with the argmin, the
// 64-bit key is key(s) << 32 | point index, so ties go to the lowest index.
constexpr unsigned int DKEY_INIT = 0xFF800000u;                 // key(+inf)
constexpr unsigned long long DKEY64_INIT = 0xFF800000FFFFFFFFull;  // (+inf, index -1)

__device__ __forceinline__ unsigned int dkey(float s) {
    const unsigned int u = __float_as_uint(s);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float dkey_value(unsigned int k) {
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}
// Signed distance sign(s) sqrt|s| of a merged key (one square root per pose).
__device__ __forceinline__ float dkey_distance(unsigned int k) {
    const float sq = dkey_value(k);
    return sq < 0.0f ? -__builtin_sqrtf(-sq) : __builtin_sqrtf(sq);
}

// One launch of the fused transform + signed distance + min-over-points
// stage: npose poses, points split into nchunk chunks of `chunk` points;
// each (pose, chunk) minimum is merged into key[g] (or key64[g]).
struct DminLaunch {
    const float4* poses;
    int npose;
    PoseTime pt;
    PointArgs pts;
    int chunk, nchunk, block;
    int kind;          // 0 polygon, 1 rectangle cover
    const float2* verts;  // polygon, padded to `padded` vertices (repeats of v0)
    const float4* rects;  // rectangle cover, padded to `padded` boxes (repeats of box 0)
    int padded;
    bool argmin;
    unsigned int* key;         // [npose], initialised to DKEY_INIT
    unsigned long long* key64; // [npose], initialised to DKEY64_INIT (argmin)
};

hipError_t launch_dmin(const DminLaunch& L, hipStream_t s);
int dmin_padded_count(int kind, int count);  // bucket a footprint size is padded to

hipError_t launch_key_init(unsigned int* key, unsigned long long* key64, int n, hipStream_t s);
hipError_t launch_dmin_finalize(const unsigned int* key, const unsigned long long* key64, int npose,
                                float* d_out, int* idx_out, hipStream_t s);

hipError_t launch_sdf_points(int kind, const float* px, const float* py, int n,
                             const float4* tab_a, const float4* tab_b, int count, float* out,
                             hipStream_t s);

hipError_t launch_compact_points(const float* x, const float* y, const float* vx, const float* vy,
                                 const unsigned char* valid, int n, float* ox, float* oy,
                                 float* ovx, float* ovy, int* oidx, int* n_valid, hipStream_t s);

struct RolloutOut {
    const float* useq = nullptr;  // [K][T][nu] given control sequences (no noise), or nullptr
    float* eps_ws;   // [T][nu][Kpad] (may be nullptr with useq)
    float4* poses;   // [T][Kpad]
    float* jbase;    // [Kpad]
    unsigned int* key;          // [T][Kpad] distance keys to initialise (or nullptr)
    unsigned long long* key64;  // [T][Kpad] (argmin variant, or nullptr)
    float* diag_poses;  // [K][T][4] or nullptr
    float* diag_eps;    // [K][T][nu]
    float* diag_u;      // [K][T][nu]
};

hipError_t launch_rollout(const StepArgs& P, const float* U, const RolloutOut& o, hipStream_t s);

hipError_t launch_cost(const StepArgs& P, const unsigned int* key, const unsigned long long* key64,
                       const float* jbase, float* jt, float* diag_dmin, int* diag_argmin,
                       hipStream_t s);

hipError_t launch_update(const StepArgs& P, const float* jt, const float* eps_ws, const float* U,
                         float* Unew, float* diag_w, hipStream_t s);

hipError_t launch_nominal(const StepArgs& P, const float* Unew, float4* nom_poses,
                          unsigned int* key_nom, hipStream_t s);

hipError_t launch_finalize(const StepArgs& P, int validate, const unsigned int* key_nom,
                           const float4* nom, const float* Unew, float* U, float* out,
                           float* diag_unew, float* diag_dnom, float* diag_jnom, hipStream_t s);

// Small steps (the single-scene path): cost + update in one launch when
// cost_update_fused(Kpad, T), and nominal + validation distances +
// validation in one single-workgroup launch when the footprint needs one lane
// per pose (polygons of up to 16 vertices, rectangle covers) and T N
// (padded primitives) <= VAL_SMALL_MAX_PAIRS.  Bit-identical to the separate
// launches.
constexpr int COST_UPDATE_MAX_KPAD = 512;               // LDS: 21 Kpad floats' worth
constexpr long long COST_UPDATE_MAX_POSES = 1ll << 15;  // Kpad T: every workgroup decodes them all
inline bool cost_update_fused(int Kpad, int T) {
    return Kpad <= COST_UPDATE_MAX_KPAD && static_cast<long long>(Kpad) * T <= COST_UPDATE_MAX_POSES;
}
constexpr int VAL_SMALL_THREADS = 1024;
constexpr long long VAL_SMALL_MAX_PAIRS = 1ll << 18;
hipError_t launch_cost_update(const StepArgs& P, const unsigned int* key,
                              const unsigned long long* key64, const float* jbase,
                              const float* eps_ws, const float* U, float* Unew, float* jt,
                              float* diag_w, float* diag_dmin, int* diag_argmin, hipStream_t s);
bool validate_small_supported(int kind, int padded);
hipError_t launch_validate_small(const StepArgs& P, int kind, int padded, const PointArgs& pts,
                                 const float2* verts, const float4* rects, const float* Unew,
                                 float* U, float* out, float* diag_unew, float* diag_dnom,
                                 float* diag_jnom, hipStream_t s);

// ---------------------------------------------------------------- batched path
// Per-step arguments of one scene (refreshed by one host-to-device copy per
// step, so a captured graph replays with new poses, seeds and nominals).
struct SceneStep {
    StepArgs P;
    float* U;  // the scene's T x nu nominal (device), updated in place
};

// Static per-scene workspaces.
struct SceneBufs {
    float* eps_ws;   // [T][nu][Kpad]
    float4* poses;   // [T][Kpad]
    float* jbase;    // [Kpad]
    float* jt;       // [Kpad]
    unsigned int* key;      // [T*Kpad] distance keys
    float* unew;     // [T][nu]
    float4* nom;     // [T]
    unsigned int* key_nom;  // [T]
    float* out;      // OUT_FLOATS floats
    int validate;    // run Algorithm 1 step 4 for this scene
};

// One (scene, pass) for the persistent signed-distance kernel.
struct SceneDmin {
    const float4* poses;
    int npose;
    PoseTime pt;
    PointArgs pts;
    int chunk;
    int kind, padded;
    const float2* verts;
    const float4* rects;
    unsigned int* key;
};

// One work item: pose tile [g0, g0 + blockDim) of SceneDmin sd against the
// compacted points [c0, c1) (clipped to the valid count on the device).
struct DminItem {
    int sd, g0, c0, c1;
};

// Register class of a footprint bucket (padded primitive count) in the
// persistent kernel, each compiled for the occupancy its largest bucket
// allows without spilling in the point loop: 0 polygons of 3..8 vertices
// (6 waves per SIMD), 1 polygons of 9..16 (4 waves), 2 polygons padded to
// 18..30 with a lane pair per pose (4 waves), 3 polygons padded to 32 with a
// lane pair per pose (3 waves), 4 rectangle covers up to 12 boxes (8
// waves), 5 larger covers (2 waves), 6 polygons padded to 36..64 with a lane
// quad per pose (3 waves).
constexpr int DMIN_CLASSES = 7;
inline int dmin_class(int kind, int padded) {
    if (kind == 1) return padded <= 12 ? 4 : 5;
    return padded <= 8 ? 0 : padded <= 16 ? 1 : padded <= 30 ? 2 : padded <= 32 ? 3 : 6;
}
// Lanes that share one pose in a register class.
constexpr int dmin_class_lanes(int cls) { return cls == 2 || cls == 3 ? 2 : cls == 6 ? 4 : 1; }

hipError_t launch_batch_reset(int* counters, int n, hipStream_t s);
hipError_t launch_rollout_batched(const SceneStep* steps, const SceneBufs* bufs, const int2* blk,
                                  int nblk, hipStream_t s);
hipError_t launch_dmin_persistent(int cls, int block, int grid, const SceneDmin* sds,
                                  const DminItem* items, int n_items, int* counter, hipStream_t s);
hipError_t launch_cost_batched(const SceneStep* steps, const SceneBufs* bufs, const int2* blk,
                               int nblk, hipStream_t s);
hipError_t launch_update_batched(const SceneStep* steps, const SceneBufs* bufs, const int2* blk,
                                 int nblk, hipStream_t s);
hipError_t launch_nominal_batched(const SceneStep* steps, const SceneBufs* bufs, int n,
                                  hipStream_t s);
hipError_t launch_finalize_batched(const SceneStep* steps, const SceneBufs* bufs, int n,
                                   hipStream_t s);
// Diagnostics of one scene of the last batched step in the caller's [r][h]
// layouts (any output may be nullptr): d_min decoded from the merged keys,
// scored poses, clipped perturbations, J~, the updated nominal, d_nom
// (validation pass) and J_nom.
struct SceneDiag {
    float *d_min, *poses, *eps, *J, *U_upd, *d_nom, *J_nom;
};
hipError_t launch_scene_diag(const SceneBufs& B, int K, int Kpad, int T, int nu,
                             const SceneDiag& d, hipStream_t s);
// Workgroups of k_dmin_persistent<cls> (block threads) resident per compute
// unit on the current device, from the occupancy calculator (registers and
// the LDS tile); 0 on error.
int dmin_persistent_blocks_per_cu(int cls, int block);
int dmin_persistent_lanes_per_pose(int cls);

// ---------------------------------------------------------------- hybrid modes
constexpr int HYB_MAX_MODES = 8;

// Mode selection and actuator post-processing of one hybrid-mode cycle
// (Algorithm 2, steps 2 and 3), from the per-mode result records.
struct HybridArgs {
    int n_modes, m_prev, tau_cool, cool_max;
    float lambda_switch, v_min, w_min, noise_v, noise_w;
    int model[HYB_MAX_MODES];
    int nu[HYB_MAX_MODES];
};

// res = (u*_0, u*_1, u*_2, m*, tau_cool', safe_stop, Jbar(m*), 0).
hipError_t launch_hybrid_select(const float* out, const HybridArgs& a, float* res, hipStream_t s);

}  // namespace emppi
