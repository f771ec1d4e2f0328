// Single-scene kernels of the sampling + rollout, cost, path-integral update,
// nominal re-rollout and validation stages (Algorithm 1 steps 1, 2-3, 4).
// The per-workgroup work is in step_device.hpp (shared with the batched
// kernels).
#include "step_device.hpp"

namespace emppi {

namespace {

__global__ __launch_bounds__(ROLL_THREADS) void k_rollout(StepArgs P, const float* __restrict__ U,
                                                 RolloutOut o) {
    __shared__ float lds[ROLL_LDS_FLOATS];
    rollout_block(P, U, o, blockIdx.x * WAVE, lds);
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

}  // namespace

hipError_t launch_rollout(const StepArgs& P, const float* U, const RolloutOut& o, hipStream_t s) {
    hipLaunchKernelGGL(k_rollout, dim3(P.Kpad / WAVE), dim3(ROLL_THREADS), 0, s, P, U, o);
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
