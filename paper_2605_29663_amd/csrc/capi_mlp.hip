// C ABI of the learned sampling proposal (declared in include/exact_mppi.h):
// parameters, features, forward pass, training step (hand-written forward and
// backward GEMMs on the matrix cores, Adam), save / load.
#include <cstdio>

#include "ctx.hpp"
#include "mlp.hpp"

using namespace emppi;
using namespace emppi_host;

struct mppi_proposal_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    int T = 0, nu = 0, in = 0, H = 0, out = 0, max_batch = 0;
    long long n_params = 0;
    long long off[6] = {0};  // W1, b1, W2, b2, W3, b3 in the flat parameter vector
    DevBuf w, g, m, v;       // fp32 master parameters, gradients, Adam moments
    DevBuf w1b, w2b, w3b;    // bf16 weight copies
    DevBuf xb, pre1, a1b, pre2, a2b, outb, dout, doutb, dh2, dh2b, dh1, dh1b, rowsq, loss;
    float* h_loss = nullptr;  // pinned
    long long t = 0;          // Adam step
    FeatArgs F{};
};

namespace {

int pfail(mppi_proposal p, int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (p)
        p->err = buf;
    else
        g_create_error = buf;
    return code;
}

#define PHIP(p, expr)                                                                         \
    do {                                                                                      \
        hipError_t _e = (expr);                                                               \
        if (_e != hipSuccess)                                                                 \
            return pfail((p), MPPI_E_HIP, "%s failed: %s", #expr, hipGetErrorString(_e));     \
    } while (0)

float* W(mppi_proposal p, DevBuf& b, int k) { return b.as<float>() + p->off[k]; }

int refresh_bf16(mppi_proposal p) {
    PHIP(p, launch_f32_to_bf16(W(p, p->w, 0), p->w1b.as<uint16_t>(), (long)p->in * p->H, p->stream));
    PHIP(p, launch_f32_to_bf16(W(p, p->w, 2), p->w2b.as<uint16_t>(), (long)p->H * p->H, p->stream));
    PHIP(p, launch_f32_to_bf16(W(p, p->w, 4), p->w3b.as<uint16_t>(), (long)p->H * p->out, p->stream));
    return MPPI_OK;
}

GemmArgs gemm(int M, int N, int K, const void* A, long sam, long sak, const void* B, long sbk,
              long sbn, float* C, void* Cb, long ldc, const float* bias, const float* aux, int epi) {
    GemmArgs g;
    g.M = M;
    g.N = N;
    g.K = K;
    g.A = static_cast<const uint16_t*>(A);
    g.sam = sam;
    g.sak = sak;
    g.B = static_cast<const uint16_t*>(B);
    g.sbk = sbk;
    g.sbn = sbn;
    g.C = C;
    g.Cb = static_cast<uint16_t*>(Cb);
    g.ldc = ldc;
    g.bias = bias;
    g.aux = aux;
    g.epi = epi;
    return g;
}

// Forward pass of M feature rows (device fp32, M x in) into p->outb (M x out).
int forward(mppi_proposal p, const float* dfeat, int M) {
    const int in = p->in, H = p->H, O = p->out;
    PHIP(p, launch_to_bf16_padded(dfeat, M, in, in, p->xb.as<uint16_t>(), in, p->stream));
    PHIP(p, launch_gemm(gemm(M, H, in, p->xb.p, in, 1, p->w1b.p, H, 1, p->pre1.as<float>(), p->a1b.p, H,
                             W(p, p->w, 1), nullptr, EPI_BIAS_GELU), p->stream));
    PHIP(p, launch_gemm(gemm(M, H, H, p->a1b.p, H, 1, p->w2b.p, H, 1, p->pre2.as<float>(), p->a2b.p, H,
                             W(p, p->w, 3), nullptr, EPI_BIAS_GELU), p->stream));
    PHIP(p, launch_gemm(gemm(M, O, H, p->a2b.p, H, 1, p->w3b.p, O, 1, p->outb.as<float>(), nullptr, O,
                             W(p, p->w, 5), nullptr, EPI_BIAS), p->stream));
    return MPPI_OK;
}

int check_batch(mppi_proposal p, int M) {
    if (M < 1 || M > p->max_batch) return pfail(p, MPPI_E_CAPACITY, "batch %d outside [1, %d]", M, p->max_batch);
    return MPPI_OK;
}

}  // namespace

extern "C" {

int proposal_create(mppi_proposal* out, int device, void* hip_stream, int T, int nu, int hidden,
                    int max_batch) {
    if (!out) return pfail(nullptr, MPPI_E_ARG, "out is NULL");
    *out = nullptr;
    if (T < 1 || T > MPPI_MAX_T || nu < 1 || nu > 3 || hidden < 1 || hidden > 4096 || max_batch < 1 ||
        max_batch > (1 << 20))
        return pfail(nullptr, MPPI_E_CAPACITY, "bad proposal shape");
    mppi_proposal p = new mppi_proposal_s;
    p->device = device;
    p->stream = static_cast<hipStream_t>(hip_stream);
    p->T = T;
    p->nu = nu;
    p->in = FEAT_BINS + 2 + T * nu;
    p->H = hidden;
    p->out = T * nu;
    p->max_batch = max_batch;
    const long long sizes[6] = {(long long)p->in * hidden, hidden, (long long)hidden * hidden, hidden,
                                (long long)hidden * p->out, p->out};
    long long acc = 0;
    for (int k = 0; k < 6; ++k) {
        p->off[k] = acc;
        acc += sizes[k];
    }
    p->n_params = acc;
    p->F.T = T;
    p->F.nu = nu;
    p->F.in_dim = p->in;
    p->F.r_max = 8.0f;
    for (int c = 0; c < 3; ++c) {
        p->F.umin[c] = -1.0f;
        p->F.umax[c] = 1.0f;
    }
    DeviceGuard g(device);
    const size_t P = sizeof(float) * acc, MB = max_batch;
    hipError_t e = hipSuccess;
    DevBuf* f32[] = {&p->w, &p->g, &p->m, &p->v};
    for (DevBuf* b : f32)
        if (e == hipSuccess) e = b->ensure(P);
    if (e == hipSuccess) e = p->w1b.ensure(2 * sizes[0]);
    if (e == hipSuccess) e = p->w2b.ensure(2 * sizes[2]);
    if (e == hipSuccess) e = p->w3b.ensure(2 * sizes[4]);
    if (e == hipSuccess) e = p->xb.ensure(2 * MB * p->in);
    if (e == hipSuccess) e = p->pre1.ensure(4 * MB * hidden);
    if (e == hipSuccess) e = p->a1b.ensure(2 * MB * hidden);
    if (e == hipSuccess) e = p->pre2.ensure(4 * MB * hidden);
    if (e == hipSuccess) e = p->a2b.ensure(2 * MB * hidden);
    if (e == hipSuccess) e = p->outb.ensure(4 * MB * p->out);
    if (e == hipSuccess) e = p->dout.ensure(4 * MB * p->out);
    if (e == hipSuccess) e = p->doutb.ensure(2 * MB * p->out);
    if (e == hipSuccess) e = p->dh2.ensure(4 * MB * hidden);
    if (e == hipSuccess) e = p->dh2b.ensure(2 * MB * hidden);
    if (e == hipSuccess) e = p->dh1.ensure(4 * MB * hidden);
    if (e == hipSuccess) e = p->dh1b.ensure(2 * MB * hidden);
    if (e == hipSuccess) e = p->rowsq.ensure(4 * MB);
    if (e == hipSuccess) e = p->loss.ensure(4);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&p->h_loss), sizeof(float), 0);
    if (e == hipSuccess) e = hipMemsetAsync(p->w.p, 0, P, p->stream);
    if (e == hipSuccess) e = hipMemsetAsync(p->m.p, 0, P, p->stream);
    if (e == hipSuccess) e = hipMemsetAsync(p->v.p, 0, P, p->stream);
    // the matrix-core copies of the (zero) weights must be valid before any forward pass
    if (e == hipSuccess && refresh_bf16(p) != MPPI_OK) e = hipErrorLaunchFailure;
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) {
        proposal_destroy(p);
        return pfail(nullptr, MPPI_E_HIP, "proposal setup: %s", hipGetErrorString(e));
    }
    *out = p;
    return MPPI_OK;
}

int proposal_destroy(mppi_proposal p) {
    if (!p) return MPPI_OK;
    {
        DeviceGuard g(p->device);
        (void)hipStreamSynchronize(p->stream);
        DevBuf* bufs[] = {&p->w, &p->g, &p->m, &p->v, &p->w1b, &p->w2b, &p->w3b, &p->xb, &p->pre1,
                          &p->a1b, &p->pre2, &p->a2b, &p->outb, &p->dout, &p->doutb, &p->dh2,
                          &p->dh2b, &p->dh1, &p->dh1b, &p->rowsq, &p->loss};
        for (DevBuf* b : bufs) b->release();
        if (p->h_loss) (void)hipHostFree(p->h_loss);
    }
    delete p;
    return MPPI_OK;
}

const char* proposal_last_error(mppi_proposal p) { return p ? p->err.c_str() : g_create_error.c_str(); }

long long proposal_num_params(mppi_proposal p) { return p ? p->n_params : -1; }

int proposal_shape(mppi_proposal p, int* in_dim, int* hidden, int* out_dim) {
    if (!p) return MPPI_E_ARG;
    if (in_dim) *in_dim = p->in;
    if (hidden) *hidden = p->H;
    if (out_dim) *out_dim = p->out;
    return MPPI_OK;
}

int proposal_set_params(mppi_proposal p, const float* host, long long n) {
    if (!p || !host) return MPPI_E_ARG;
    if (n != p->n_params) return pfail(p, MPPI_E_ARG, "expected %lld parameters", p->n_params);
    DeviceGuard g(p->device);
    PHIP(p, hipMemcpyAsync(p->w.p, host, sizeof(float) * n, hipMemcpyHostToDevice, p->stream));
    PHIP(p, hipMemsetAsync(p->m.p, 0, sizeof(float) * n, p->stream));
    PHIP(p, hipMemsetAsync(p->v.p, 0, sizeof(float) * n, p->stream));
    p->t = 0;
    if (int rc = refresh_bf16(p)) return rc;
    PHIP(p, hipStreamSynchronize(p->stream));
    return MPPI_OK;
}

int proposal_get_params(mppi_proposal p, float* host, long long n) {
    if (!p || !host) return MPPI_E_ARG;
    if (n != p->n_params) return pfail(p, MPPI_E_ARG, "expected %lld parameters", p->n_params);
    DeviceGuard g(p->device);
    PHIP(p, hipMemcpyAsync(host, p->w.p, sizeof(float) * n, hipMemcpyDeviceToHost, p->stream));
    PHIP(p, hipStreamSynchronize(p->stream));
    return MPPI_OK;
}

int proposal_set_scaling(mppi_proposal p, const mppi_params* prm, float r_max) {
    if (!p || !prm) return MPPI_E_ARG;
    if (prm->T != p->T || prm->nu != p->nu) return pfail(p, MPPI_E_ARG, "T / nu differ from the proposal's");
    if (!(r_max > 0)) return pfail(p, MPPI_E_ARG, "r_max must be positive");
    p->F.r_max = r_max;
    p->F.goal[0] = prm->goal[0];
    p->F.goal[1] = prm->goal[1];
    for (int c = 0; c < 3; ++c) {
        p->F.umin[c] = c < prm->nu ? prm->u_min[c] : -1.0f;
        p->F.umax[c] = c < prm->nu ? prm->u_max[c] : 1.0f;
    }
    return MPPI_OK;
}

int proposal_features(mppi_proposal p, mppi_ctx ctx, const float* dq0, const float* dU_prev, int M,
                      float* dfeat) {
    if (!p || !ctx || !dq0 || !dU_prev || !dfeat) return MPPI_E_ARG;
    if (M < 1) return pfail(p, MPPI_E_ARG, "M < 1");
    DeviceGuard g(p->device);
    PHIP(p, launch_features(ctx->px.as<float>(), ctx->py.as<float>(), ctx->n_valid.as<int>(), dq0,
                            dU_prev, p->F, M, dfeat, p->stream));
    return MPPI_OK;
}

int proposal_forward(mppi_proposal p, const float* dfeat, int M, float* dout) {
    if (!p || !dfeat || !dout) return MPPI_E_ARG;
    if (int rc = check_batch(p, M)) return rc;
    DeviceGuard g(p->device);
    if (int rc = forward(p, dfeat, M)) return rc;
    PHIP(p, hipMemcpyAsync(dout, p->outb.p, sizeof(float) * M * p->out, hipMemcpyDeviceToDevice, p->stream));
    return MPPI_OK;
}

int proposal_mean(mppi_proposal p, const float* dfeat, int M, float* dU) {
    if (!p || !dfeat || !dU) return MPPI_E_ARG;
    if (int rc = check_batch(p, M)) return rc;
    DeviceGuard g(p->device);
    if (int rc = forward(p, dfeat, M)) return rc;
    PHIP(p, launch_denorm(p->outb.as<float>(), dfeat, M, p->T, p->nu, p->F, dU, p->stream));
    return MPPI_OK;
}

int proposal_normalize(mppi_proposal p, const float* dU, const float* dfeat, int M, float* dtarget) {
    if (!p || !dU || !dtarget) return MPPI_E_ARG;
    if (M < 1) return pfail(p, MPPI_E_ARG, "M < 1");
    if (p->F.res_scale > 0.0f && !dfeat) return pfail(p, MPPI_E_ARG, "residual targets need the features");
    DeviceGuard g(p->device);
    PHIP(p, launch_normalize(dU, dfeat, M, p->T, p->nu, p->F, dtarget, p->stream));
    return MPPI_OK;
}

int proposal_set_residual(mppi_proposal p, float scale) {
    if (!p) return MPPI_E_ARG;
    if (!(scale >= 0.0f) || !std::isfinite(scale)) return pfail(p, MPPI_E_ARG, "scale must be >= 0");
    p->F.res_scale = scale;
    return MPPI_OK;
}

int proposal_train_step(mppi_proposal p, const float* dfeat, const float* dtarget, int M, float lr,
                        float* loss_out) {
    if (!p || !dfeat || !dtarget) return MPPI_E_ARG;
    if (int rc = check_batch(p, M)) return rc;
    if (!(lr >= 0)) return pfail(p, MPPI_E_ARG, "lr must be >= 0");
    DeviceGuard g(p->device);
    const int in = p->in, H = p->H, O = p->out;
    if (int rc = forward(p, dfeat, M)) return rc;
    PHIP(p, launch_mse_grad(p->outb.as<float>(), dtarget, M, O, p->dout.as<float>(), p->doutb.as<uint16_t>(),
                            p->rowsq.as<float>(), p->loss.as<float>(), p->stream));
    // layer 3: dW3 = A2^T dOut, db3 = sum dOut, dH2 = (dOut W3^T) * gelu'(pre2)
    PHIP(p, launch_gemm(gemm(H, O, M, p->a2b.p, 1, H, p->doutb.p, O, 1, W(p, p->g, 4), nullptr, O, nullptr,
                             nullptr, EPI_STORE), p->stream));
    PHIP(p, launch_colsum(p->dout.as<float>(), M, O, W(p, p->g, 5), p->stream));
    PHIP(p, launch_gemm(gemm(M, H, O, p->doutb.p, O, 1, p->w3b.p, 1, O, p->dh2.as<float>(), p->dh2b.p, H,
                             nullptr, p->pre2.as<float>(), EPI_GELU_GRAD), p->stream));
    // layer 2
    PHIP(p, launch_gemm(gemm(H, H, M, p->a1b.p, 1, H, p->dh2b.p, H, 1, W(p, p->g, 2), nullptr, H, nullptr,
                             nullptr, EPI_STORE), p->stream));
    PHIP(p, launch_colsum(p->dh2.as<float>(), M, H, W(p, p->g, 3), p->stream));
    PHIP(p, launch_gemm(gemm(M, H, H, p->dh2b.p, H, 1, p->w2b.p, 1, H, p->dh1.as<float>(), p->dh1b.p, H,
                             nullptr, p->pre1.as<float>(), EPI_GELU_GRAD), p->stream));
    // layer 1
    PHIP(p, launch_gemm(gemm(in, H, M, p->xb.p, 1, in, p->dh1b.p, H, 1, W(p, p->g, 0), nullptr, H, nullptr,
                             nullptr, EPI_STORE), p->stream));
    PHIP(p, launch_colsum(p->dh1.as<float>(), M, H, W(p, p->g, 1), p->stream));
    // Adam
    p->t += 1;
    AdamArgs a;
    a.lr = lr;
    a.b1 = 0.9f;
    a.b2 = 0.999f;
    a.ob1 = static_cast<float>(1.0 - 0.9);
    a.ob2 = static_cast<float>(1.0 - 0.999);
    a.eps = 1e-8f;
    a.c1 = static_cast<float>(1.0 - std::pow(0.9, static_cast<double>(p->t)));
    a.c2 = static_cast<float>(1.0 - std::pow(0.999, static_cast<double>(p->t)));
    PHIP(p, launch_adam(p->w.as<float>(), p->g.as<float>(), p->m.as<float>(), p->v.as<float>(), p->n_params,
                        a, p->stream));
    if (int rc = refresh_bf16(p)) return rc;
    if (loss_out) {
        PHIP(p, hipMemcpyAsync(p->h_loss, p->loss.p, sizeof(float), hipMemcpyDeviceToHost, p->stream));
        PHIP(p, hipStreamSynchronize(p->stream));
        *loss_out = *p->h_loss;
    }
    return MPPI_OK;
}

int proposal_get_buffer(mppi_proposal p, int which, float* host, long long n) {
    if (!p || !host) return MPPI_E_ARG;
    DeviceGuard g(p->device);
    DevBuf* f32[] = {&p->pre1, &p->pre2, &p->outb, &p->dout, &p->dh2, &p->dh1, &p->g};
    DevBuf* b16[] = {&p->xb, &p->a1b, &p->a2b, &p->doutb, &p->dh2b, &p->dh1b};
    if (which >= 0 && which < 7) {
        if (static_cast<size_t>(n) * 4 > f32[which]->cap) return pfail(p, MPPI_E_ARG, "n too large");
        PHIP(p, hipMemcpyAsync(host, f32[which]->p, sizeof(float) * n, hipMemcpyDeviceToHost, p->stream));
        PHIP(p, hipStreamSynchronize(p->stream));
        return MPPI_OK;
    }
    if (which >= 10 && which < 16) {
        DevBuf* b = b16[which - 10];
        if (static_cast<size_t>(n) * 2 > b->cap) return pfail(p, MPPI_E_ARG, "n too large");
        std::vector<uint16_t> tmp(n);
        PHIP(p, hipMemcpyAsync(tmp.data(), b->p, 2 * n, hipMemcpyDeviceToHost, p->stream));
        PHIP(p, hipStreamSynchronize(p->stream));
        for (long long i = 0; i < n; ++i) {
            const uint32_t u = static_cast<uint32_t>(tmp[i]) << 16;
            std::memcpy(&host[i], &u, 4);
        }
        return MPPI_OK;
    }
    return pfail(p, MPPI_E_ARG, "unknown buffer %d", which);
}

int proposal_save(mppi_proposal p, const char* path) {
    if (!p || !path) return MPPI_E_ARG;
    std::vector<float> w(p->n_params), m(p->n_params), v(p->n_params);
    DeviceGuard g(p->device);
    PHIP(p, hipMemcpyAsync(w.data(), p->w.p, 4 * p->n_params, hipMemcpyDeviceToHost, p->stream));
    PHIP(p, hipMemcpyAsync(m.data(), p->m.p, 4 * p->n_params, hipMemcpyDeviceToHost, p->stream));
    PHIP(p, hipMemcpyAsync(v.data(), p->v.p, 4 * p->n_params, hipMemcpyDeviceToHost, p->stream));
    PHIP(p, hipStreamSynchronize(p->stream));
    FILE* f = std::fopen(path, "wb");
    if (!f) return pfail(p, MPPI_E_ARG, "cannot open %s", path);
    const int hdr[6] = {0x50494d46, p->in, p->H, p->out, p->T, p->nu};  // "EMIP"
    bool ok = std::fwrite(hdr, sizeof hdr, 1, f) == 1 && std::fwrite(&p->t, sizeof p->t, 1, f) == 1 &&
              std::fwrite(&p->F, sizeof p->F, 1, f) == 1 &&
              std::fwrite(w.data(), 4, w.size(), f) == w.size() &&
              std::fwrite(m.data(), 4, m.size(), f) == m.size() &&
              std::fwrite(v.data(), 4, v.size(), f) == v.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? MPPI_OK : pfail(p, MPPI_E_ARG, "write failed: %s", path);
}

int proposal_load(mppi_proposal p, const char* path) {
    if (!p || !path) return MPPI_E_ARG;
    FILE* f = std::fopen(path, "rb");
    if (!f) return pfail(p, MPPI_E_ARG, "cannot open %s", path);
    int hdr[6];
    long long t = 0;
    FeatArgs F;
    std::vector<float> w(p->n_params), m(p->n_params), v(p->n_params);
    bool ok = std::fread(hdr, sizeof hdr, 1, f) == 1 && hdr[0] == 0x50494d46 && hdr[1] == p->in &&
              hdr[2] == p->H && hdr[3] == p->out && std::fread(&t, sizeof t, 1, f) == 1 &&
              std::fread(&F, sizeof F, 1, f) == 1 && std::fread(w.data(), 4, w.size(), f) == w.size() &&
              std::fread(m.data(), 4, m.size(), f) == m.size() &&
              std::fread(v.data(), 4, v.size(), f) == v.size();
    std::fclose(f);
    if (!ok) return pfail(p, MPPI_E_ARG, "%s is not a proposal of this shape", path);
    DeviceGuard g(p->device);
    PHIP(p, hipMemcpyAsync(p->w.p, w.data(), 4 * p->n_params, hipMemcpyHostToDevice, p->stream));
    PHIP(p, hipMemcpyAsync(p->m.p, m.data(), 4 * p->n_params, hipMemcpyHostToDevice, p->stream));
    PHIP(p, hipMemcpyAsync(p->v.p, v.data(), 4 * p->n_params, hipMemcpyHostToDevice, p->stream));
    p->t = t;
    p->F = F;
    if (int rc = refresh_bf16(p)) return rc;
    PHIP(p, hipStreamSynchronize(p->stream));
    return MPPI_OK;
}

}  // extern "C"
