// Internal interface of the learned-proposal kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace emppi {

constexpr int FEAT_BINS = 64;  // polar range histogram bins

// Feature / output scaling of one proposal.
struct FeatArgs {
    int T, nu, in_dim;
    float r_max;             // histogram range clip (m); also scales the goal
    float goal[2];
    float umin[3], umax[3];  // control box: features and outputs use (u - mid) / half
    float res_scale;         // > 0: the output is a residual on the previous sequence
};

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_GRAD = 3 };

struct GemmArgs {
    int M, N, K;
    const uint16_t* A;  // bf16 bits
    long sam, sak;
    const uint16_t* B;
    long sbk, sbn;
    float* C;           // fp32 output (pre-activation / gradient)
    uint16_t* Cb;       // bf16 output (activation / gradient), EPI_BIAS_GELU and EPI_GELU_GRAD
    long ldc;
    const float* bias;  // EPI_BIAS, EPI_BIAS_GELU
    const float* aux;   // EPI_GELU_GRAD: pre-activation, same layout as C
    int epi;
};

struct AdamArgs {
    // decay rates b1, b2 and their complements ob1 = 1 - b1, ob2 = 1 - b2 (formed in
    // double, so that at t = 1 the moment scale and the bias correction cancel exactly);
    // c1 = 1 - b1^t, c2 = 1 - b2^t
    float lr, b1, b2, ob1, ob2, eps, c1, c2;
};

hipError_t launch_features(const float* px, const float* py, const int* n_valid, const float* q0s,
                           const float* U_prev, const FeatArgs& F, int n_states, float* feat,
                           hipStream_t s);
hipError_t launch_to_bf16_padded(const float* src, int rows, int cols, int ld_src, uint16_t* dst,
                                 int ld_dst, hipStream_t s);
hipError_t launch_gemm(const GemmArgs& g, hipStream_t s);
hipError_t launch_mse_grad(const float* out, const float* tgt, int M, int n_out, float* dout,
                           uint16_t* dout_b, float* row_sq, float* loss, hipStream_t s);
hipError_t launch_colsum(const float* d, int M, int N, float* out, hipStream_t s);
hipError_t launch_adam(float* w, const float* grad, float* m, float* v, long n, const AdamArgs& a,
                       hipStream_t s);
hipError_t launch_f32_to_bf16(const float* src, uint16_t* dst, long n, hipStream_t s);
hipError_t launch_normalize(const float* U, const float* feat, int M, int T, int nu, const FeatArgs& F, float* y,
                            hipStream_t s);
hipError_t launch_denorm(const float* y, const float* feat, int M, int T, int nu, const FeatArgs& F, float* U,
                         hipStream_t s);

}  // namespace emppi
