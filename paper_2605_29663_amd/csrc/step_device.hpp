// Device building blocks of the sampling / rollout, cost, update, nominal and
// validation stages (Algorithm 1 steps 1, 2-3, 4), shared by the
// single-scene kernels and the batched ones.  Every reduction has a fixed
// order, so a scene gives bit-identical results whether it runs alone or in
// a batch, eagerly or from a captured graph.
#pragma once
#include "devmath.hpp"
#include "kernels.hpp"

namespace emppi {

constexpr int ROLL_HCHUNK = 16;                   // horizon steps per rollout chunk
constexpr int ROLL_THREADS = WAVE * ROLL_HCHUNK;  // one (rollout, step) pair per thread
// LDS of a rollout workgroup of rb rollouts, per (step, rollout) pair: the
// heading rate / heading / task terms, (cos, sin) of the heading, and the
// planar velocity / position.
constexpr int roll_lds_floats(int rb, int hc = ROLL_HCHUNK) { return 5 * rb * hc; }
constexpr int ROLL_LDS_FLOATS = roll_lds_floats(WAVE);
// Rollouts per workgroup of the single-scene rollout kernel when K is small:
// 16 rollouts x 16 steps = 256 threads, four times as many workgroups (and
// compute units) as 64-rollout blocks, the same per-pair arithmetic.
constexpr int ROLL_RB_SMALL = 16;
constexpr int COST_THREADS = 1024;  // 64 rollouts x 16 horizon groups
constexpr int FIN_THREADS = 128;    // one thread per horizon step
constexpr int NOM_THREADS = 128;    // one thread per horizon step
constexpr int NOM_LDS_FLOATS = 5 * MPPI_MAX_T_DEV;

// One forward-Euler step q_{h+1} = q_h + F_m(q_h, u_h) dt (Section "Robot
// Kinematic Models") in the fixed single-precision sequence, split into the
// heading recursion theta_{h+1} = theta_h + omega(u_h) dt (which does not
// depend on the position) and the position recursion p_{h+1} = p_h +
// v(u_h, theta_h) dt, where the planar velocity v uses (s, c) = sin / cos of
// theta_h.  "a += b dt" is one fma(b, dt, a).  Splitting them lets the
// costly sin / cos and tan and the velocities of every step run in parallel,
// while each serial recursion is a chain of fmas on values read into
// registers ahead of it; the values are those of a plain step-by-step
// integration.
__device__ __forceinline__ bool model_rotates(int model) { return model <= 3; }
__device__ __forceinline__ bool model_translates(int model) { return model != 3; }

__device__ __forceinline__ float heading_rate(int model, const float u[3], float L) {
    switch (model) {
    case 0: return u[1];                        // unicycle (v, omega)
    case 1: return (u[0] * seq_tan(u[1])) / L;  // Ackermann (v, delta): v tan(delta) / L
    case 2: return u[2];                        // omni (vx, vy, omega)
    case 3: return u[0];                        // spin in place (omega)
    default: return 0.0f;                       // parallel: heading held
    }
}

// Planar velocity of a translating model at heading (s, c) = (sin, cos).
__device__ __forceinline__ float2 planar_velocity(int model, const float u[3], float s, float c) {
    switch (model) {
    case 0:
    case 1: return make_float2(u[0] * c, u[0] * s);
    case 2: return make_float2(__builtin_fmaf(u[0], c, -(u[1] * s)), __builtin_fmaf(u[0], s, u[1] * c));
    default: return make_float2(-(u[0] * s), u[0] * c);  // parallel: along the body y axis
    }
}

// Serial recursions over n <= HC steps whose per-step inputs sit in
// LDS at a[k * stride] (k < n): every input is read into a register first,
// then the fma chain runs and each state is written back over its input.  A
// full chunk (n == HC) runs straight-line code; a partial one (the
// horizon's last chunk) a short loop.
template <int HC = ROLL_HCHUNK>
__device__ __forceinline__ float heading_chain(float* a, int stride, int n, float dt, float th) {
    if (n == HC) {
        float w[HC];
#pragma unroll
        for (int k = 0; k < HC; ++k) w[k] = a[k * stride];
#pragma unroll
        for (int k = 0; k < HC; ++k) {
            th = __builtin_fmaf(w[k], dt, th);
            a[k * stride] = th;
        }
    } else {
        for (int k = 0; k < n; ++k) {
            th = __builtin_fmaf(a[k * stride], dt, th);
            a[k * stride] = th;
        }
    }
    return th;
}

template <int HC = ROLL_HCHUNK>
__device__ __forceinline__ void position_chain(float2* a, int stride, int n, float dt, float& x,
                                               float& y) {
    if (n == HC) {
        float2 v[HC];
#pragma unroll
        for (int k = 0; k < HC; ++k) v[k] = a[k * stride];
#pragma unroll
        for (int k = 0; k < HC; ++k) {
            x = __builtin_fmaf(v[k].x, dt, x);
            y = __builtin_fmaf(v[k].y, dt, y);
            a[k * stride] = make_float2(x, y);
        }
    } else {
        for (int k = 0; k < n; ++k) {
            const float2 v = a[k * stride];
            x = __builtin_fmaf(v.x, dt, x);
            y = __builtin_fmaf(v.y, dt, y);
            a[k * stride] = make_float2(x, y);
        }
    }
}

template <int HC = ROLL_HCHUNK>
__device__ __forceinline__ float sum_chain(const float* a, int stride, int n, float acc) {
    if (n == HC) {
        float w[HC];
#pragma unroll
        for (int k = 0; k < HC; ++k) w[k] = a[k * stride];
#pragma unroll
        for (int k = 0; k < HC; ++k) acc += w[k];
    } else {
        for (int k = 0; k < n; ++k) acc += a[k * stride];
    }
    return acc;
}

// Distance of (px, py) to the guidance polyline: min over its segments of
// the clipped-projection point-segment distance (one waypoint: the distance
// to it).
__device__ __forceinline__ float path_dist(const float2* __restrict__ path, int n, float px,
                                           float py) {
    float2 a = path[0];
    float best = (px - a.x) * (px - a.x) + (py - a.y) * (py - a.y);
    for (int k = 1; k < n; ++k) {
        const float2 b = path[k];
        const float ex = b.x - a.x, ey = b.y - a.y;
        const float wx = px - a.x, wy = py - a.y;
        const float ee = ex * ex + ey * ey;
        float t = ee > 0.0f ? (wx * ex + wy * ey) / ee : 0.0f;
        t = fminf(fmaxf(t, 0.0f), 1.0f);
        const float rx = wx - t * ex, ry = wy - t * ey;
        best = fminf(best, rx * rx + ry * ry);
        a = b;
    }
    return __builtin_sqrtf(best);
}

// Task + control terms of one scored state (the obstacle term is added once
// the signed distances exist): goal distance, guidance-path distance and the
// control regulariser.
__device__ __forceinline__ float task_ctrl(const StepArgs& P, float px, float py, const float u[3]) {
    const float gx = px - P.goal[0], gy = py - P.goal[1];
    float v = P.w_goal * __builtin_sqrtf(gx * gx + gy * gy);
    if (P.n_path > 0) v += P.w_path * path_dist(P.path, P.n_path, px, py);
    for (int c = 0; c < P.nu; ++c) v += P.w_ctrl[c] * (u[c] * u[c]);
    return v;
}

// Sampling + rollouts of rollouts [r0, r0 + RB) (Algorithm 1 step 1), by
// chunks of HC horizon steps with RB * HC threads; thread
// (step hh, rollout l) keeps its pair's control in registers:
//   (a) every thread draws the noise of its pair, clamps the sampled control
//       and evaluates its heading rate;
//   (b) the first RB threads (hh = 0), one per rollout: the heading
//       recursion;
//   (c) every thread: sin / cos of its pair's new heading, then (d) the
//       planar velocity at the heading before its step;
//   (e) the first RB threads: the position recursion;
//   (f) every thread: its pair's scored pose, the distance keys' initial
//       values and the task + control terms, which the first RB threads then
//       add up in step order.
// The result depends on neither RB nor HC.  lds: roll_lds_floats(RB, HC)
// floats.
template <int RB = WAVE, int HC = ROLL_HCHUNK>
__device__ __forceinline__ void rollout_block(const StepArgs& P, const float* __restrict__ U,
                                              const RolloutOut& o, int r0, float* lds) {
    const int T = P.T, nu = P.nu, Kpad = P.Kpad;
    float* sw = lds;  // [hh][lane] heading rate, then heading, then task + control terms
    float2* scs = reinterpret_cast<float2*>(lds + RB * HC);      // [hh][lane] (c, s) after step
    float2* sxy = reinterpret_cast<float2*>(lds + 3 * RB * HC);  // [hh][lane] velocity, then position after step
    const int lane = threadIdx.x % RB, hh = threadIdx.x / RB;
    const int r = r0 + lane;
    const bool chain = threadIdx.x < RB;  // hh == 0
    const bool rotates = model_rotates(P.model), translates = model_translates(P.model);
    // chain threads: the state at the start of the chunk
    float x = P.q0[0], y = P.q0[1], th = P.q0[2], s = 0.f, c = 1.f, jb = 0.0f;
    if (chain) seq_sincos(th, s, c);
    for (int h0 = 0; h0 < T; h0 += HC) {
        const int hn = min(HC, T - h0);
        const int h = h0 + hh;
        const bool act = hh < hn;
        float u[3] = {0.f, 0.f, 0.f};
        if (act) {
            if (r < P.K && o.useq) {
                // a given sequence, clamped to the control box, no noise
                for (int k = 0; k < nu; ++k) {
                    float v = o.useq[(static_cast<size_t>(r) * T + h) * nu + k];
                    v = fmaxf(v, P.umin[k]);
                    u[k] = fminf(v, P.umax[k]);
                }
            } else if (r < P.K) {
                float ub[3] = {0.f, 0.f, 0.f};  // issued ahead of the noise arithmetic
                for (int k = 0; k < nu; ++k) ub[k] = U[h * nu + k];
                float z[4];
                normals4(P.seed, P.step, static_cast<uint32_t>(r), static_cast<uint32_t>(h), P.stream, z);
                for (int k = 0; k < nu; ++k) {
                    const float base = ub[k];
                    float v = base + P.sigma[k] * z[k];
                    v = fmaxf(v, P.umin[k]);
                    v = fminf(v, P.umax[k]);
                    const float e = v - base;
                    u[k] = v;
                    o.eps_ws[(h * nu + k) * Kpad + r] = e;
                    const size_t d = (static_cast<size_t>(r) * T + h) * nu + k;
                    if (o.diag_eps) o.diag_eps[d] = e;
                    if (o.diag_u) o.diag_u[d] = v;
                }
            } else if (o.eps_ws) {
                // padding rollouts [K, Kpad): weight exp(-inf) = 0 in the
                // update, which multiplies these entries, so they must hold a
                // finite value (0 * NaN left over in reused memory is NaN)
                for (int k = 0; k < nu; ++k) o.eps_ws[(h * nu + k) * Kpad + r] = 0.0f;
            }
            sw[hh * RB + lane] = heading_rate(P.model, u, P.wheelbase);
        }
        __syncthreads();
        if (chain) {
            if (rotates) {
                th = heading_chain<HC>(sw + lane, RB, hn, P.dt, th);
            } else {
                for (int k = 0; k < hn; ++k) sw[k * RB + lane] = th;
            }
        }
        __syncthreads();
        float cn = 1.f, sn = 0.f;
        if (act) {
            seq_sincos(sw[hh * RB + lane], sn, cn);
            scs[hh * RB + lane] = make_float2(cn, sn);
        }
        __syncthreads();
        // heading before the step: the chain's state for hh = 0
        float cb = c, sb = s;
        if (act && hh > 0) {
            const float2 p = scs[(hh - 1) * RB + lane];
            cb = p.x;
            sb = p.y;
        }
        if (act && translates) sxy[hh * RB + lane] = planar_velocity(P.model, u, sb, cb);
        __syncthreads();
        const float xs = x, ys = y;
        if (chain) {
            if (translates) {
                position_chain<HC>(sxy + lane, RB, hn, P.dt, x, y);
            } else {
                for (int k = 0; k < hn; ++k) sxy[k * RB + lane] = make_float2(x, y);
            }
            const float2 e = scs[(hn - 1) * RB + lane];
            c = e.x;
            s = e.y;
        }
        __syncthreads();
        if (act) {
            float4 pose;
            if (P.state_offset) {
                const float2 p = sxy[hh * RB + lane];
                pose = make_float4(p.x, p.y, cn, sn);
            } else if (hh > 0) {
                const float2 p = sxy[(hh - 1) * RB + lane];
                pose = make_float4(p.x, p.y, cb, sb);
            } else {
                pose = make_float4(xs, ys, cb, sb);
            }
            o.poses[h * Kpad + r] = pose;
            if (o.key) o.key[h * Kpad + r] = DKEY_INIT;
            if (o.key64) o.key64[h * Kpad + r] = DKEY64_INIT;
            if (o.diag_poses && r < P.K) {
                float* dp = o.diag_poses + (static_cast<size_t>(r) * T + h) * 4;
                dp[0] = pose.x;
                dp[1] = pose.y;
                dp[2] = pose.z;
                dp[3] = pose.w;
            }
            sw[hh * RB + lane] = task_ctrl(P, pose.x, pose.y, u);
        }
        __syncthreads();
        if (chain) jb = sum_chain<HC>(sw + lane, RB, hn, jb);
        __syncthreads();
    }
    if (chain) o.jbase[r] = jb;
}

// J~ of rollouts [r0, r0 + 64) (Algorithm 1 steps 2-3): lane l, group q of
// the 1024 threads decodes the minimum of (r0 + l, h) for h = q, q + 16, ...,
// adds the obstacle penalties and the unsafe flag; the 16 partial sums are
// added in index order.  lds: 2 * 1024 words.
__device__ __forceinline__ void cost_block(const StepArgs& P, const unsigned int* __restrict__ key,
                                           const unsigned long long* __restrict__ key64,
                                           const float* __restrict__ jbase, float* __restrict__ jt,
                                           float* __restrict__ diag_dmin,
                                           int* __restrict__ diag_argmin, int r0, float* lds) {
    const int lane = threadIdx.x & (WAVE - 1), grp = threadIdx.x / WAVE;
    const int ngrp = blockDim.x / WAVE;
    const int r = r0 + lane;
    float J = 0.0f;
    int chi = 0;
    if (r < P.K) {
        for (int h = grp; h < P.T; h += ngrp) {
            const size_t g = static_cast<size_t>(h) * P.Kpad + r;
            float d;
            int idx = -1;
            if (key64) {
                const unsigned long long k = key64[g];
                d = dkey_distance(static_cast<unsigned int>(k >> 32));
                idx = static_cast<int>(static_cast<unsigned int>(k));
            } else {
                d = dkey_distance(key[g]);
            }
            const float gap = fmaxf(P.d_safe - d, 0.0f);
            J += (d < 0.0f ? P.w_coll : 0.0f) + P.w_rep * (gap * gap);
            chi |= (d < P.d_safe) ? 1 : 0;
            if (diag_dmin) diag_dmin[static_cast<size_t>(r) * P.T + h] = d;
            if (diag_argmin) diag_argmin[static_cast<size_t>(r) * P.T + h] = idx;
        }
    }
    float* sJ = lds;
    int* sC = reinterpret_cast<int*>(lds + COST_THREADS);
    sJ[threadIdx.x] = J;
    sC[threadIdx.x] = chi;
    __syncthreads();
    if (grp == 0 && r < P.Kpad) {
        if (r >= P.K) {
            jt[r] = INFINITY;
        } else {
            float acc = jbase[r];
            int any = 0;
            for (int q = 0; q < ngrp; ++q) {
                acc += sJ[q * WAVE + lane];
                any |= sC[q * WAVE + lane];
            }
            jt[r] = acc + (any ? P.w_inf : 0.0f);
        }
    }
}

// Deterministic block reductions (fixed butterfly within a wave, waves
// combined in index order).  sh: 16 floats.
// nw: the waves whose values are combined (every thread of the block must
// call it; the block has at most 16 waves).
template <typename Op>
__device__ __forceinline__ float block_reduce(float v, float* sh, Op op, int nw) {
    for (int o = WAVE / 2; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o));
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    __syncthreads();
    if (lane == 0) sh[wid] = v;
    __syncthreads();
    float r = sh[0];
    for (int w = 1; w < nw; ++w) r = op(r, sh[w]);
    return r;
}
template <typename Op>
__device__ __forceinline__ float block_reduce(float v, float* sh, Op op) {
    return block_reduce(v, sh, op, static_cast<int>(blockDim.x / WAVE));
}

// Horizon step h of the path-integral update (Algorithm 1 step 3):
// beta = min J~, omega = exp(-(J~ - beta)/lambda), U_h += (sum omega eps_h) /
// (sum omega).  The first NT threads do the work (NT = 0: every thread of the
// 256-thread block); every (scene, h) workgroup computes the same beta and
// normaliser in the same order.
template <int NT = 0>
__device__ __forceinline__ void update_block(const StepArgs& P, const float* __restrict__ jt,
                                             const float* __restrict__ eps_ws,
                                             const float* __restrict__ U, float* __restrict__ Unew,
                                             float* __restrict__ diag_w, int h, float* sh) {
    const int Kpad = P.Kpad, nu = P.nu;
    const int nt = NT ? NT : static_cast<int>(blockDim.x);
    const bool on = static_cast<int>(threadIdx.x) < nt;
    float b = INFINITY;
    if (on)
        for (int r = threadIdx.x; r < Kpad; r += nt) b = fminf(b, jt[r]);
    const float beta = block_reduce(b, sh, [](float a, float c) { return fminf(a, c); }, nt / WAVE);
    float z = 0.f, n0 = 0.f, n1 = 0.f, n2 = 0.f;
    const float* e0 = eps_ws + (h * nu) * Kpad;
    if (on)
        for (int r = threadIdx.x; r < Kpad; r += nt) {
            const float w = expf((beta - jt[r]) / P.lambda);
            z += w;
            n0 += w * e0[r];
            if (nu > 1) n1 += w * e0[Kpad + r];
            if (nu > 2) n2 += w * e0[2 * Kpad + r];
        }
    auto add = [](float a, float c) { return a + c; };
    const float Z = block_reduce(z, sh, add, nt / WAVE);
    const float N0 = block_reduce(n0, sh, add, nt / WAVE);
    const float N1 = nu > 1 ? block_reduce(n1, sh, add, nt / WAVE) : 0.f;
    const float N2 = nu > 2 ? block_reduce(n2, sh, add, nt / WAVE) : 0.f;
    if (threadIdx.x == 0) {
        Unew[h * nu] = U[h * nu] + N0 / Z;
        if (nu > 1) Unew[h * nu + 1] = U[h * nu + 1] + N1 / Z;
        if (nu > 2) Unew[h * nu + 2] = U[h * nu + 2] + N2 / Z;
    }
    if (diag_w && h == 0 && on)
        for (int r = threadIdx.x; r < P.K; r += nt) diag_w[r] = expf((beta - jt[r]) / P.lambda) / Z;
}

// Cost and update fused for small K (one launch instead of two), with
// COST_THREADS threads: every (horizon step h) workgroup first computes J~ of
// all Kpad rollouts in cost_block's layout and operation order (thread (lane,
// group q) sums the terms h' = q, q + 16, ... of rollout r0 + lane for every
// 64-rollout slab r0; then per rollout the task and control terms plus the 16
// partial sums in q order), so the bits are cost_block's; workgroup 0 also
// stores them to jt and writes the d_min / argmin diagnostics; then the first
// 256 threads run update_block for step h (the bits of the 256-thread
// update).  LDS: sP 16 Kpad floats, sC 16 Kpad bytes, sJ Kpad floats.
__device__ __forceinline__ void cost_update_block(const StepArgs& P,
                                                  const unsigned int* __restrict__ key,
                                                  const unsigned long long* __restrict__ key64,
                                                  const float* __restrict__ jbase,
                                                  const float* __restrict__ eps_ws,
                                                  const float* __restrict__ U,
                                                  float* __restrict__ Unew, float* __restrict__ jt,
                                                  float* __restrict__ diag_w,
                                                  float* __restrict__ diag_dmin,
                                                  int* __restrict__ diag_argmin, int h, float* sP,
                                                  unsigned char* sC, float* sJ, float* sh) {
    constexpr int NGRP = COST_THREADS / WAVE;
    const int lane = threadIdx.x & (WAVE - 1), grp = threadIdx.x / WAVE;
    const int Kpad = P.Kpad;
    const bool first = h == 0;
    // one rollout's obstacle terms and unsafe flag, term by term in h order
    auto term = [&](float d, float& J, int& chi) {
        const float gap = fmaxf(P.d_safe - d, 0.0f);
        J += (d < 0.0f ? P.w_coll : 0.0f) + P.w_rep * (gap * gap);
        chi |= (d < P.d_safe) ? 1 : 0;
    };
    if (!key64) {
        // every key this thread decodes (slab s, term i: rollout s 64 + lane,
        // step grp + 16 i) is read before the first is used, one round trip
        // to memory instead of one per key; same sums in the same order
        constexpr int NSLAB = COST_UPDATE_MAX_KPAD / WAVE;
        constexpr int NTERM = (MPPI_MAX_T_DEV + NGRP - 1) / NGRP;
        unsigned int kv[NSLAB][NTERM];
#pragma unroll
        for (int sl = 0; sl < NSLAB; ++sl)
#pragma unroll
            for (int i = 0; i < NTERM; ++i) {
                const int r = sl * WAVE + lane, hh = grp + i * NGRP;
                kv[sl][i] = DKEY_INIT;
                if (sl * WAVE < Kpad && r < P.K && hh < P.T) kv[sl][i] = key[hh * Kpad + r];
            }
#pragma unroll
        for (int sl = 0; sl < NSLAB; ++sl) {
            if (sl * WAVE >= Kpad) break;
            const int r = sl * WAVE + lane;
            float J = 0.0f;
            int chi = 0;
            if (r < P.K) {
#pragma unroll
                for (int i = 0; i < NTERM; ++i) {
                    const int hh = grp + i * NGRP;
                    if (hh >= P.T) break;
                    const float d = dkey_distance(kv[sl][i]);
                    term(d, J, chi);
                    if (first && diag_dmin) diag_dmin[static_cast<size_t>(r) * P.T + hh] = d;
                    if (first && diag_argmin) diag_argmin[static_cast<size_t>(r) * P.T + hh] = -1;
                }
            }
            sP[grp * Kpad + r] = J;
            sC[grp * Kpad + r] = static_cast<unsigned char>(chi);
        }
    } else {
        for (int r0 = 0; r0 < Kpad; r0 += WAVE) {
            const int r = r0 + lane;
            float J = 0.0f;
            int chi = 0;
            if (r < P.K) {
                for (int hh = grp; hh < P.T; hh += NGRP) {
                    const unsigned long long k = key64[static_cast<size_t>(hh) * Kpad + r];
                    const float d = dkey_distance(static_cast<unsigned int>(k >> 32));
                    term(d, J, chi);
                    if (first && diag_dmin) diag_dmin[static_cast<size_t>(r) * P.T + hh] = d;
                    if (first && diag_argmin)
                        diag_argmin[static_cast<size_t>(r) * P.T + hh] = static_cast<int>(static_cast<unsigned int>(k));
                }
            }
            sP[grp * Kpad + r] = J;
            sC[grp * Kpad + r] = static_cast<unsigned char>(chi);
        }
    }
    __syncthreads();
    for (int r = threadIdx.x; r < Kpad; r += blockDim.x) {
        float j;
        if (r >= P.K) {
            j = INFINITY;
        } else {
            float acc = jbase[r];
            int any = 0;
            for (int q = 0; q < NGRP; ++q) {
                acc += sP[q * Kpad + r];
                any |= sC[q * Kpad + r];
            }
            j = acc + (any ? P.w_inf : 0.0f);
        }
        sJ[r] = j;
        if (first) jt[r] = j;
    }
    __syncthreads();
    update_block<256>(P, sJ, eps_ws, U, Unew, diag_w, h, sh);
}

// Nominal trajectory of the updated sequence (Algorithm 1 step 4) in the same
// single-precision sequence as the sampled rollouts, with NOM_THREADS threads
// (thread h = horizon step h, holding u_h): heading rates in parallel, the
// heading recursion on thread 0, sin / cos and the planar velocities in
// parallel, the position recursion on thread 0 (both recursions in chunks
// of ROLL_HCHUNK steps read into registers), the poses in parallel.  The
// distance keys of the T nominal poses are initialised on the way.  Every
// thread returns after the poses are written (no barrier after them).
// lds: NOM_LDS_FLOATS floats.
__device__ __forceinline__ void nominal_block(const StepArgs& P, const float* __restrict__ Unew,
                                              float4* __restrict__ nom,
                                              unsigned int* __restrict__ key_nom, float* lds) {
    const int T = P.T, nu = P.nu, h = threadIdx.x;
    const bool act = h < T;
    float* sw = lds;                                                     // heading rate, then heading after step h
    float2* scs = reinterpret_cast<float2*>(lds + MPPI_MAX_T_DEV);      // (c, s) after step h
    float2* sxy = reinterpret_cast<float2*>(lds + 3 * MPPI_MAX_T_DEV);  // velocity, then position after step h
    float u[3] = {0.f, 0.f, 0.f};
    if (act) {
        for (int k = 0; k < nu; ++k) u[k] = Unew[h * nu + k];
        sw[h] = heading_rate(P.model, u, P.wheelbase);
        key_nom[h] = DKEY_INIT;
    }
    __syncthreads();
    if (h == 0) {
        float th = P.q0[2];
        for (int k0 = 0; k0 < T; k0 += ROLL_HCHUNK) {
            const int n = min(ROLL_HCHUNK, T - k0);
            if (model_rotates(P.model))
                th = heading_chain(sw + k0, 1, n, P.dt, th);
            else
                for (int k = 0; k < n; ++k) sw[k0 + k] = th;
        }
    }
    __syncthreads();
    float cn = 1.f, sn = 0.f;
    if (act) {
        seq_sincos(sw[h], sn, cn);
        scs[h] = make_float2(cn, sn);
    }
    __syncthreads();
    float cb, sb;  // heading before step h
    if (h == 0) {
        seq_sincos(P.q0[2], sb, cb);
    } else if (act) {
        const float2 p = scs[h - 1];
        cb = p.x;
        sb = p.y;
    }
    const bool translates = model_translates(P.model);
    if (act && translates) sxy[h] = planar_velocity(P.model, u, sb, cb);
    __syncthreads();
    if (h == 0) {
        float x = P.q0[0], y = P.q0[1];
        for (int k0 = 0; k0 < T; k0 += ROLL_HCHUNK) {
            const int n = min(ROLL_HCHUNK, T - k0);
            if (translates)
                position_chain(sxy + k0, 1, n, P.dt, x, y);
            else
                for (int k = 0; k < n; ++k) sxy[k0 + k] = make_float2(x, y);
        }
    }
    __syncthreads();
    if (act) {
        if (P.state_offset) {
            const float2 p = sxy[h];
            nom[h] = make_float4(p.x, p.y, cn, sn);
        } else if (h > 0) {
            const float2 p = sxy[h - 1];
            nom[h] = make_float4(p.x, p.y, cb, sb);
        } else {
            nom[h] = make_float4(P.q0[0], P.q0[1], cb, sb);
        }
    }
}

// Validation and execution (Algorithm 1 step 4): valid iff every
// d_nom >= d_safe and every control of the nominal is finite; then u* = U_0
// and U shifts left (last entry repeated), else u* = 0 and U = 0.  The noise-free cost of the updated nominal, J_nom =
// sum_h [phi_task + phi_ctrl + phi_obs] along the validation rollout (+ w_inf
// if unsafe), is what the hybrid-mode selection compares across modes.
// out = (u*_0, u*_1, u*_2, valid, J_nom, 0, 0, 0).  One thread per horizon
// step (FIN_THREADS threads); sh: 16 floats.
__device__ __forceinline__ void finalize_block(const StepArgs& P, int validate,
                                               const unsigned int* __restrict__ key_nom,
                                               const float4* __restrict__ nom,
                                               const float* __restrict__ Unew,
                                               float* __restrict__ U, float* __restrict__ out,
                                               float* __restrict__ diag_unew,
                                               float* __restrict__ diag_dnom,
                                               float* __restrict__ diag_jnom, float* sh) {
    const int T = P.T, nu = P.nu, h = threadIdx.x;
    int bad = 0;
    float term = 0.0f;
    if (validate && h < T) {
        const float d = dkey_distance(key_nom[h]);
        bad = !(d >= P.d_safe);
        if (diag_dnom) diag_dnom[h] = d;
        float u[3] = {0.f, 0.f, 0.f};
        for (int k = 0; k < nu; ++k) u[k] = Unew[h * nu + k];
        // a non-finite control has no defined trajectory: never valid (its
        // poses are NaN, and NaN distances never lower the running minimum)
        for (int k = 0; k < nu; ++k) bad |= !__builtin_isfinite(u[k]);
        const float4 p = nom[h];
        const float gap = fmaxf(P.d_safe - d, 0.0f);
        term = task_ctrl(P, p.x, p.y, u) + ((d < 0.0f ? P.w_coll : 0.0f) + P.w_rep * (gap * gap));
    }
    const int ok = !__syncthreads_or(bad);
    const float jsum = block_reduce(term, sh, [](float a, float c) { return a + c; });
    if (h < T) {
        const int src = (h + 1 < T ? h + 1 : T - 1) * nu;
        for (int k = 0; k < nu; ++k) {
            if (diag_unew) diag_unew[h * nu + k] = Unew[h * nu + k];
            U[h * nu + k] = ok ? Unew[src + k] : 0.0f;
        }
    }
    if (h == 0) {
        const float jn = validate ? jsum + (ok ? 0.0f : P.w_inf) : NAN;
        for (int k = 0; k < 3; ++k) out[k] = (ok && k < nu) ? Unew[k] : 0.0f;
        out[3] = ok ? 1.0f : 0.0f;
        out[4] = jn;
        for (int k = 5; k < OUT_FLOATS; ++k) out[k] = 0.0f;
        if (diag_jnom) diag_jnom[0] = jn;
    }
}

}  // namespace emppi
