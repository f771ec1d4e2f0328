// Sampling + rollout, cost, path-integral update, nominal re-rollout and
// validation kernels of one control cycle (Algorithm 1 steps 1, 2-3, 4).
#include "devmath.hpp"
#include "kernels.hpp"

namespace emppi {

namespace {

// One forward-Euler step q_{h+1} = q_h + F_m(q_h, u_h) dt (Section "Robot
// Kinematic Models") in the fixed single-precision sequence; (s, c) =
// sin/cos of theta_h.  "a += b dt" is one fma(b, dt, a).
__device__ __forceinline__ void euler_step(int model, const float u[3], float dt, float L, float s,
                                           float c, float& x, float& y, float& th) {
    switch (model) {
    case 0:  // unicycle (v, omega)
        x = __builtin_fmaf(u[0] * c, dt, x);
        y = __builtin_fmaf(u[0] * s, dt, y);
        th = __builtin_fmaf(u[1], dt, th);
        break;
    case 1: {  // Ackermann (v, delta): theta' = v tan(delta) / L
        const float w = (u[0] * seq_tan(u[1])) / L;
        x = __builtin_fmaf(u[0] * c, dt, x);
        y = __builtin_fmaf(u[0] * s, dt, y);
        th = __builtin_fmaf(w, dt, th);
        break;
    }
    case 2: {  // omni (vx, vy, omega)
        const float xd = __builtin_fmaf(u[0], c, -(u[1] * s));
        const float yd = __builtin_fmaf(u[0], s, u[1] * c);
        x = __builtin_fmaf(xd, dt, x);
        y = __builtin_fmaf(yd, dt, y);
        th = __builtin_fmaf(u[2], dt, th);
        break;
    }
    case 3:  // spin in place (omega)
        th = __builtin_fmaf(u[0], dt, th);
        break;
    default:  // parallel (v_para)
        x = __builtin_fmaf(-(u[0] * s), dt, x);
        y = __builtin_fmaf(u[0] * c, dt, y);
        break;
    }
}

// Task + control terms of one scored state (the obstacle term is added by
// k_cost once the signed distances exist).
__device__ __forceinline__ float task_ctrl(const StepArgs& P, float px, float py, const float u[3]) {
    const float gx = px - P.goal[0], gy = py - P.goal[1];
    float v = P.w_goal * __fsqrt_rn(gx * gx + gy * gy);
    for (int c = 0; c < P.nu; ++c) v += P.w_ctrl[c] * (u[c] * u[c]);
    return v;
}

// Phase 1: the noise of all (r, h) of a 64-rollout tile, in parallel over
// the workgroup; phase 2: one wave integrates the 64 rollouts over h.
__global__ __launch_bounds__(256) void k_rollout(StepArgs P, const float* __restrict__ U,
                                                 float* __restrict__ u_ws, RolloutOut o) {
    const int r0 = blockIdx.x * WAVE;
    const int T = P.T, nu = P.nu, Kpad = P.Kpad;
    for (int p = threadIdx.x; p < WAVE * T; p += blockDim.x) {
        const int r = r0 + (p & (WAVE - 1)), h = p / WAVE;
        if (r >= P.K) continue;
        float z[4];
        normals4(P.seed, P.step, static_cast<uint32_t>(r), static_cast<uint32_t>(h), P.stream, z);
        for (int c = 0; c < nu; ++c) {
            const float base = U[h * nu + c];
            float v = base + P.sigma[c] * z[c];
            v = fmaxf(v, P.umin[c]);
            v = fminf(v, P.umax[c]);
            const float e = v - base;
            o.eps_ws[(h * nu + c) * Kpad + r] = e;
            u_ws[(h * nu + c) * Kpad + r] = v;
            const size_t d = (static_cast<size_t>(r) * T + h) * nu + c;
            if (o.diag_eps) o.diag_eps[d] = e;
            if (o.diag_u) o.diag_u[d] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x >= WAVE) return;
    const int r = r0 + threadIdx.x;
    const bool live = r < P.K;
    float x = P.q0[0], y = P.q0[1], th = P.q0[2], s, c;
    seq_sincos(th, s, c);
    float jb = 0.0f;
    for (int h = 0; h < T; ++h) {
        float u[3] = {0.f, 0.f, 0.f};
        if (live)
            for (int k = 0; k < nu; ++k) u[k] = u_ws[(h * nu + k) * Kpad + r];
        float4 pose = make_float4(x, y, c, s);
        euler_step(P.model, u, P.dt, P.wheelbase, s, c, x, y, th);
        seq_sincos(th, s, c);
        if (P.state_offset) pose = make_float4(x, y, c, s);
        o.poses[h * Kpad + r] = pose;
        if (o.diag_poses && live)
            reinterpret_cast<float4*>(o.diag_poses)[static_cast<size_t>(r) * T + h] = pose;
        jb += task_ctrl(P, pose.x, pose.y, u);
    }
    o.jbase[r] = jb;
}

// J~ per rollout: task/control sum + obstacle penalty over h, unsafe flag.
__global__ __launch_bounds__(256) void k_cost(StepArgs P, const float* __restrict__ part,
                                              const int* __restrict__ part_idx, int nchunk,
                                              const float* __restrict__ jbase,
                                              float* __restrict__ jt,
                                              float* __restrict__ diag_dmin,
                                              int* __restrict__ diag_argmin) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= P.Kpad) return;
    if (r >= P.K) {
        jt[r] = INFINITY;
        return;
    }
    const size_t npose = static_cast<size_t>(P.T) * P.Kpad;
    float J = jbase[r];
    bool chi = false;
    for (int h = 0; h < P.T; ++h) {
        const size_t g = static_cast<size_t>(h) * P.Kpad + r;
        float sq = part[g];
        int idx = part_idx ? part_idx[g] : -1;
        for (int c = 1; c < nchunk; ++c) {
            const float v = part[c * npose + g];
            if (v < sq) {
                sq = v;
                if (part_idx) idx = part_idx[c * npose + g];
            }
        }
        const float d = sq < 0.0f ? -__fsqrt_rn(-sq) : __fsqrt_rn(sq);
        const float gap = fmaxf(P.d_safe - d, 0.0f);
        J += (d < 0.0f ? P.w_coll : 0.0f) + P.w_rep * (gap * gap);
        chi = chi || (d < P.d_safe);
        if (diag_dmin) diag_dmin[static_cast<size_t>(r) * P.T + h] = d;
        if (diag_argmin) diag_argmin[static_cast<size_t>(r) * P.T + h] = idx;
    }
    jt[r] = J + (chi ? P.w_inf : 0.0f);
}

// Deterministic block reductions (fixed butterfly within a wave, waves
// combined in index order).
template <typename Op>
__device__ __forceinline__ float block_reduce(float v, float* sh, Op op) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    float r = sh[0];
    for (int w = 1; w < static_cast<int>(blockDim.x / WAVE); ++w) r = op(r, sh[w]);
    return r;
}

// One workgroup per horizon step h: beta = min J~, omega = exp(-(J~-beta)/lambda),
// U_h <- U_h + (sum omega eps_h) / (sum omega).  Every workgroup computes the
// same beta and normaliser in the same order.
__global__ __launch_bounds__(256) void k_update(StepArgs P, const float* __restrict__ jt,
                                                const float* __restrict__ eps_ws,
                                                const float* __restrict__ U,
                                                float* __restrict__ Unew,
                                                float* __restrict__ diag_w) {
    __shared__ float sh[16];
    const int h = blockIdx.x;
    const int Kpad = P.Kpad, nu = P.nu;
    float b = INFINITY;
    for (int r = threadIdx.x; r < Kpad; r += blockDim.x) b = fminf(b, jt[r]);
    const float beta = block_reduce(b, sh, [](float a, float c) { return fminf(a, c); });
    float z = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f;
    const float* e0 = eps_ws + (h * nu) * Kpad;
    for (int r = threadIdx.x; r < Kpad; r += blockDim.x) {
        const float w = expf((beta - jt[r]) / P.lambda);
        z += w;
        n0 += w * e0[r];
        if (nu > 1) n1 += w * e0[Kpad + r];
        if (nu > 2) n2 += w * e0[2 * Kpad + r];
    }
    auto add = [](float a, float c) { return a + c; };
    const float Z = block_reduce(z, sh, add);
    const float N0 = block_reduce(n0, sh, add);
    const float N1 = nu > 1 ? block_reduce(n1, sh, add) : 0.f;
    const float N2 = nu > 2 ? block_reduce(n2, sh, add) : 0.f;
    if (threadIdx.x == 0) {
        Unew[h * nu] = U[h * nu] + N0 / Z;
        if (nu > 1) Unew[h * nu + 1] = U[h * nu + 1] + N1 / Z;
        if (nu > 2) Unew[h * nu + 2] = U[h * nu + 2] + N2 / Z;
    }
    if (diag_w && h == 0)
        for (int r = threadIdx.x; r < P.K; r += blockDim.x)
            diag_w[r] = expf((beta - jt[r]) / P.lambda) / Z;
}

// Nominal trajectory of the updated sequence (Algorithm 1 step 4), same
// single-precision sequence as the sampled rollouts.
__global__ void k_nominal(StepArgs P, const float* __restrict__ Unew, float4* __restrict__ nom) {
    if (threadIdx.x != 0) return;
    float x = P.q0[0], y = P.q0[1], th = P.q0[2], s, c;
    seq_sincos(th, s, c);
    for (int h = 0; h < P.T; ++h) {
        float u[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < P.nu; ++k) u[k] = Unew[h * P.nu + k];
        float4 pose = make_float4(x, y, c, s);
        euler_step(P.model, u, P.dt, P.wheelbase, s, c, x, y, th);
        seq_sincos(th, s, c);
        if (P.state_offset) pose = make_float4(x, y, c, s);
        nom[h] = pose;
    }
}

// Validation and execution: valid iff every d_nom >= d_safe; then u* = U_0
// and U shifts left (last entry repeated), else u* = 0 and U = 0.
// out4 = (u*_0, u*_1, u*_2, valid).
__global__ __launch_bounds__(128) void k_finalize(StepArgs P, int validate,
                                                  const float* __restrict__ part_nom, int nchunk,
                                                  const float* __restrict__ Unew,
                                                  float* __restrict__ U, float* __restrict__ out4,
                                                  float* __restrict__ diag_unew,
                                                  float* __restrict__ diag_dnom) {
    const int h = threadIdx.x, T = P.T, nu = P.nu;
    int bad = 0;
    if (validate && h < T) {
        float sq = part_nom[h];
        for (int c = 1; c < nchunk; ++c) sq = fminf(sq, part_nom[c * T + h]);
        const float d = sq < 0.0f ? -__fsqrt_rn(-sq) : __fsqrt_rn(sq);
        bad = !(d >= P.d_safe);
        if (diag_dnom) diag_dnom[h] = d;
    }
    const int ok = !__syncthreads_or(bad);
    if (h < T) {
        const int src = (h + 1 < T ? h + 1 : T - 1) * nu;
        for (int c = 0; c < nu; ++c) {
            if (diag_unew) diag_unew[h * nu + c] = Unew[h * nu + c];
            U[h * nu + c] = ok ? Unew[src + c] : 0.0f;
        }
    }
    if (h == 0) {
        for (int c = 0; c < 3; ++c) out4[c] = (ok && c < nu) ? Unew[c] : 0.0f;
        out4[3] = ok ? 1.0f : 0.0f;
    }
}

}  // namespace

hipError_t launch_rollout(const StepArgs& P, const float* U, float* u_ws, const RolloutOut& o,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_rollout, dim3(P.Kpad / WAVE), dim3(256), 0, s, P, U, u_ws, o);
    return hipGetLastError();
}

hipError_t launch_cost(const StepArgs& P, const float* part, const int* part_idx, int nchunk,
                       const float* jbase, const int*, float* jt, float* diag_dmin,
                       int* diag_argmin, hipStream_t s) {
    hipLaunchKernelGGL(k_cost, dim3((P.Kpad + 255) / 256), dim3(256), 0, s, P, part, part_idx,
                       nchunk, jbase, jt, diag_dmin, diag_argmin);
    return hipGetLastError();
}

hipError_t launch_update(const StepArgs& P, const float* jt, const float* eps_ws, const float* U,
                         float* Unew, float* diag_w, hipStream_t s) {
    hipLaunchKernelGGL(k_update, dim3(P.T), dim3(256), 0, s, P, jt, eps_ws, U, Unew, diag_w);
    return hipGetLastError();
}

hipError_t launch_nominal(const StepArgs& P, const float* Unew, float4* nom, hipStream_t s) {
    hipLaunchKernelGGL(k_nominal, dim3(1), dim3(WAVE), 0, s, P, Unew, nom);
    return hipGetLastError();
}

hipError_t launch_finalize(const StepArgs& P, int validate, const float* part_nom, int nchunk,
                           const float* Unew, float* U, float* out4, float* diag_unew,
                           float* diag_dnom, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(128), 0, s, P, validate, part_nom, nchunk, Unew, U,
                       out4, diag_unew, diag_dnom);
    return hipGetLastError();
}

}  // namespace emppi
