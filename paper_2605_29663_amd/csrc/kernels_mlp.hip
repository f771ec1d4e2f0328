// Learned sampling proposal: feature extraction, bf16 matrix-core GEMMs with
// fused epilogues, loss, bias gradients, Adam and weight conversion.
//
// Network: features (64-bin polar range histogram, goal in the robot frame,
// previous control sequence) -> Linear -> GELU -> Linear -> GELU -> Linear ->
// mean control sequence (normalised units).  bf16 operands on the gfx950
// matrix cores (v_mfma_f32_16x16x32_bf16), fp32 accumulation, fp32 master
// weights and Adam moments.
#include "devmath.hpp"
#include "mlp.hpp"

namespace emppi {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bf16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ uint16_t to_bf16(float x) {
    const uint32_t u = __float_as_uint(x);
    return static_cast<uint16_t>((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

// GELU with the exact error function and its derivative.
__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
           x * 0.39894228040143268f * expf(-0.5f * x * x);
}

// ---------------------------------------------------------------- features
// One workgroup per state.  Points go to the robot frame at q0 (rotation by
// the single-precision sin/cos sequence), the bin is a pseudo-angle built from
// correctly rounded divisions only (quadrant q, t in [0,1], bin = 16 q +
// min(15, floor(16 t))), the range is the correctly rounded square root; the
// per-bin minimum is an LDS atomicMin on the bits of the non-negative float.
__global__ __launch_bounds__(1024) void k_features(const float* __restrict__ px,
                                                   const float* __restrict__ py,
                                                   const int* __restrict__ n_valid,
                                                   const float* __restrict__ q0s,
                                                   const float* __restrict__ U_prev, FeatArgs F,
                                                   float* __restrict__ feat) {
    __shared__ unsigned int hist[FEAT_BINS];
    const int state = blockIdx.x;
    const float* q0 = q0s + 3 * state;
    const float* Up = U_prev + static_cast<size_t>(state) * F.T * F.nu;
    float* out = feat + static_cast<size_t>(state) * F.in_dim;
    for (int b = threadIdx.x; b < FEAT_BINS; b += blockDim.x) hist[b] = __float_as_uint(F.r_max);
    __syncthreads();
    float s, c;
    seq_sincos(q0[2], s, c);
    const int nv = *n_valid;
    for (int i = threadIdx.x; i < nv; i += blockDim.x) {
        const float dx = px[i] - q0[0], dy = py[i] - q0[1];
        const float x = c * dx + s * dy;
        const float y = c * dy - s * dx;
        int q;
        float t;
        if (y >= 0.0f) {
            if (x >= 0.0f) {
                q = 0;
                t = (x == 0.0f && y == 0.0f) ? 0.0f : y / (x + y);
            } else {
                q = 1;
                t = -x / (y - x);
            }
        } else {
            if (x < 0.0f) {
                q = 2;
                t = -y / (-x - y);
            } else {
                q = 3;
                t = x / (x - y);
            }
        }
        const int bin = q * 16 + min(15, static_cast<int>(t * 16.0f));
        const float r = seq_sqrt(x * x + y * y);
        atomicMin(&hist[bin], __float_as_uint(fminf(r, F.r_max)));
    }
    __syncthreads();
    for (int b = threadIdx.x; b < FEAT_BINS; b += blockDim.x) out[b] = __uint_as_float(hist[b]) / F.r_max;
    if (threadIdx.x == 0) {
        const float gx = F.goal[0] - q0[0], gy = F.goal[1] - q0[1];
        out[FEAT_BINS] = (c * gx + s * gy) / F.r_max;
        out[FEAT_BINS + 1] = (c * gy - s * gx) / F.r_max;
    }
    for (int k = threadIdx.x; k < F.T * F.nu; k += blockDim.x) {
        const int ch = k % F.nu;
        const float mid = (F.umax[ch] + F.umin[ch]) * 0.5f;
        const float half = (F.umax[ch] - F.umin[ch]) * 0.5f;
        out[FEAT_BINS + 2 + k] = half > 0.0f ? (Up[k] - mid) / half : 0.0f;
    }
}

// ---------------------------------------------------------------- conversion
__global__ void k_to_bf16_padded(const float* __restrict__ src, int rows, int cols, int ld_src,
                                 uint16_t* __restrict__ dst, int ld_dst) {
    const int r = blockIdx.y, c = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows || c >= ld_dst) return;
    dst[static_cast<size_t>(r) * ld_dst + c] = c < cols ? to_bf16(src[static_cast<size_t>(r) * ld_src + c]) : 0;
}

// ---------------------------------------------------------------- GEMM
// C[M x N] = A[M x K] * B[K x N] with general strides (bf16 operands):
// A(m, k) = A[m * sam + k * sak], B(k, n) = B[k * sbk + n * sbn].
// Workgroup tile 64 x 64 (4 waves in 2 x 2, each 32 x 32 = 2 x 2 blocks of
// v_mfma_f32_16x16x32_bf16), K in steps of 32 through LDS, with the operands
// stored k-contiguous ([row][k] and [col][k]) so each lane reads its 8
// consecutive k values with one 16-byte load.  Lane l of a 16 x 16 x 32 MFMA
// holds A rows l % 16, k = 8 (l / 16) .. +7, B columns l % 16 with the same k,
// and D rows 4 (l / 16) .. +3 of column l % 16.
constexpr int GT = 64, GK = 32, GKP = GK + 8;  // tile, k step, padded LDS row (bf16)

__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ __attribute__((aligned(16))) uint16_t As[GT][GKP];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[GT][GKP];
    const int m0 = blockIdx.y * GT, n0 = blockIdx.x * GT;
    const int w = threadIdx.x / WAVE, l = threadIdx.x % WAVE;
    const int wm = w / 2, wn = w % 2;
    f32x4 acc[2][2];
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += GK) {
        __syncthreads();
        for (int e = threadIdx.x; e < GT * GK; e += blockDim.x) {
            const int r = e / GK, k = e % GK;
            const int m = m0 + r, n = n0 + r, kk = k0 + k;
            As[r][k] = (m < g.M && kk < g.K) ? g.A[static_cast<size_t>(m) * g.sam + static_cast<size_t>(kk) * g.sak] : 0;
            Bs[r][k] = (n < g.N && kk < g.K) ? g.B[static_cast<size_t>(kk) * g.sbk + static_cast<size_t>(n) * g.sbn] : 0;
        }
        __syncthreads();
        bf16x8 a[2], b[2];
        for (int i = 0; i < 2; ++i) {
            const int row = wm * 32 + i * 16 + (l % 16);
            a[i] = *reinterpret_cast<const bf16x8*>(&As[row][8 * (l / 16)]);
        }
        for (int j = 0; j < 2; ++j) {
            const int col = wn * 32 + j * 16 + (l % 16);
            b[j] = *reinterpret_cast<const bf16x8*>(&Bs[col][8 * (l / 16)]);
        }
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            for (int t = 0; t < 4; ++t) {
                const int m = m0 + wm * 32 + i * 16 + 4 * (l / 16) + t;
                const int n = n0 + wn * 32 + j * 16 + (l % 16);
                if (m >= g.M || n >= g.N) continue;
                const size_t o = static_cast<size_t>(m) * g.ldc + n;
                float v = acc[i][j][t];
                switch (g.epi) {
                case EPI_STORE:
                    g.C[o] = v;
                    break;
                case EPI_BIAS:
                    g.C[o] = v + g.bias[n];
                    break;
                case EPI_BIAS_GELU: {
                    const float pre = v + g.bias[n];
                    g.C[o] = pre;
                    g.Cb[o] = to_bf16(gelu(pre));
                    break;
                }
                case EPI_GELU_GRAD: {
                    const float d = v * gelu_grad(g.aux[o]);
                    g.C[o] = d;
                    g.Cb[o] = to_bf16(d);
                    break;
                }
                default:
                    break;
                }
            }
}

// ---------------------------------------------------------------- loss, bias grads
// dOut = 2 (out - target) / (M n_out) (fp32 and bf16), per-row squared error.
__global__ void k_mse_grad(const float* __restrict__ out, const float* __restrict__ tgt, int M,
                           int n_out, float* __restrict__ dout, uint16_t* __restrict__ dout_b,
                           float* __restrict__ row_sq) {
    const int m = blockIdx.x;
    float acc = 0.f;
    const float scale = 2.0f / (static_cast<float>(M) * static_cast<float>(n_out));
    for (int j = threadIdx.x; j < n_out; j += blockDim.x) {
        const size_t o = static_cast<size_t>(m) * n_out + j;
        const float e = out[o] - tgt[o];
        const float d = scale * e;
        dout[o] = d;
        dout_b[o] = to_bf16(d);
        acc += e * e;
    }
    // fixed-order block sum (binary tree; blockDim.x is 256)
    __shared__ float sh[256];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) row_sq[m] = sh[0];
}

// Loss = sum of the row sums / (M n_out), fixed order: thread t adds rows
// t, t + 1024, ... in turn, then a fixed binary tree over the 1024 partials.
constexpr int LOSS_THREADS = 1024;

__global__ __launch_bounds__(LOSS_THREADS) void k_loss_sum(const float* __restrict__ row_sq, int M,
                                                           int n_out, float* __restrict__ loss) {
    __shared__ float sh[LOSS_THREADS];
    float s = 0.f;
    for (int m = threadIdx.x; m < M; m += LOSS_THREADS) s += row_sq[m];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = LOSS_THREADS / 2; w > 0; w >>= 1) {
        if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = sh[0] / (static_cast<float>(M) * static_cast<float>(n_out));
}

// Column sums over the batch (bias gradients), fixed order: a block holds
// 64 columns (one per lane) and COLSUM_GROUPS row groups (one per wave);
// group g adds rows g, g + COLSUM_GROUPS, ... in turn, and the group
// partials are added in group order.
constexpr int COLSUM_GROUPS = 16;

__global__ __launch_bounds__(64 * COLSUM_GROUPS) void k_colsum(const float* __restrict__ d, int M, int N,
                                                               float* __restrict__ out) {
    __shared__ float sh[COLSUM_GROUPS][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + lane;
    float s = 0.f;
    if (n < N)
        for (int m = g; m < M; m += COLSUM_GROUPS) s += d[static_cast<size_t>(m) * N + n];
    sh[g][lane] = s;
    __syncthreads();
    if (g == 0 && n < N) {
        float t = sh[0][lane];
#pragma unroll
        for (int k = 1; k < COLSUM_GROUPS; ++k) t += sh[k][lane];
        out[n] = t;
    }
}

// ---------------------------------------------------------------- Adam
// w -= lr * mhat / (sqrt(vhat) + eps), mhat = m / (1 - b1^t), vhat = v / (1 - b2^t).
__global__ void k_adam(float* __restrict__ w, const float* __restrict__ grad, float* __restrict__ m,
                       float* __restrict__ v, long n, AdamArgs a) {
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float mi = a.b1 * m[i] + a.ob1 * g;
    const float vi = a.b2 * v[i] + a.ob2 * (g * g);
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / a.c1, vh = vi / a.c2;
    w[i] = w[i] - a.lr * mh / (sqrtf(vh) + a.eps);
}

__global__ void k_f32_to_bf16(const float* __restrict__ src, uint16_t* __restrict__ dst, long n) {
    const long i = static_cast<long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = to_bf16(src[i]);
}

// Normalised network output -> control sequence in the actuator box:
// u = clamp(mid + half * y, u_min, u_max) per channel.
// In residual mode (res_scale > 0) the output is added to the previous
// sequence's scaled value carried in the features: ys = feat_U + res_scale y.
__global__ void k_denorm(const float* __restrict__ y, const float* __restrict__ feat, int M, int T,
                         int nu, FeatArgs F, float* __restrict__ U) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * T * nu) return;
    const int ch = i % nu;
    const int m = i / (T * nu), k = i % (T * nu);
    const float ys = F.res_scale > 0.0f
                         ? __builtin_fmaf(F.res_scale, y[i], feat[static_cast<size_t>(m) * F.in_dim + FEAT_BINS + 2 + k])
                         : y[i];
    const float mid = (F.umax[ch] + F.umin[ch]) * 0.5f;
    const float half = (F.umax[ch] - F.umin[ch]) * 0.5f;
    U[i] = fminf(fmaxf(mid + half * ys, F.umin[ch]), F.umax[ch]);
}

// Control sequences -> normalised training targets: y = (u - mid) / half.
// (residual mode: y = (ys - feat_U) / res_scale)
__global__ void k_normalize(const float* __restrict__ U, const float* __restrict__ feat, int M,
                            int T, int nu, FeatArgs F, float* __restrict__ y) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= M * T * nu) return;
    const int ch = i % nu;
    const int m = i / (T * nu), k = i % (T * nu);
    const float mid = (F.umax[ch] + F.umin[ch]) * 0.5f;
    const float half = (F.umax[ch] - F.umin[ch]) * 0.5f;
    const float ys = half > 0.0f ? (U[i] - mid) / half : 0.0f;
    y[i] = F.res_scale > 0.0f
               ? (ys - feat[static_cast<size_t>(m) * F.in_dim + FEAT_BINS + 2 + k]) / F.res_scale
               : ys;
}

}  // namespace

hipError_t launch_normalize(const float* U, const float* feat, int M, int T, int nu,
                            const FeatArgs& F, float* y, hipStream_t s) {
    const int n = M * T * nu;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_normalize, dim3((n + 255) / 256), dim3(256), 0, s, U, feat, M, T, nu, F, y);
    return hipGetLastError();
}

hipError_t launch_features(const float* px, const float* py, const int* n_valid, const float* q0s,
                           const float* U_prev, const FeatArgs& F, int n_states, float* feat,
                           hipStream_t s) {
    if (n_states <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3(n_states), dim3(1024), 0, s, px, py, n_valid, q0s, U_prev, F,
                       feat);
    return hipGetLastError();
}

hipError_t launch_to_bf16_padded(const float* src, int rows, int cols, int ld_src, uint16_t* dst,
                                 int ld_dst, hipStream_t s) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_bf16_padded, dim3((ld_dst + 255) / 256, rows), dim3(256), 0, s, src,
                       rows, cols, ld_src, dst, ld_dst);
    return hipGetLastError();
}

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gemm, dim3((g.N + GT - 1) / GT, (g.M + GT - 1) / GT), dim3(256), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_mse_grad(const float* out, const float* tgt, int M, int n_out, float* dout,
                           uint16_t* dout_b, float* row_sq, float* loss, hipStream_t s) {
    hipLaunchKernelGGL(k_mse_grad, dim3(M), dim3(256), 0, s, out, tgt, M, n_out, dout, dout_b, row_sq);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_loss_sum, dim3(1), dim3(LOSS_THREADS), 0, s, row_sq, M, n_out, loss);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* d, int M, int N, float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3((N + 63) / 64), dim3(64 * COLSUM_GROUPS), 0, s, d, M, N, out);
    return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* grad, float* m, float* v, long n, const AdamArgs& a,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, w,
                       grad, m, v, n, a);
    return hipGetLastError();
}

hipError_t launch_f32_to_bf16(const float* src, uint16_t* dst, long n, hipStream_t s) {
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s,
                       src, dst, n);
    return hipGetLastError();
}

hipError_t launch_denorm(const float* y, const float* feat, int M, int T, int nu, const FeatArgs& F,
                         float* U, hipStream_t s) {
    const int n = M * T * nu;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_denorm, dim3((n + 255) / 256), dim3(256), 0, s, y, feat, M, T, nu, F, U);
    return hipGetLastError();
}

}  // namespace emppi
