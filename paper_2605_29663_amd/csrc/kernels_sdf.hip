// Fused rollout-frame transform + exact signed distance + min over points
// (the hot stage of one MPPI step), the point-wise signed-distance kernels,
// and the obstacle-point compaction that implements the validity mask.
//
// Paper: Section "Signed Distance Evaluation" (rollout-frame transform,
// box distance, polygon distance with ray-casting sign) and Section "Batched
// Rollout and Distance Computation" (K x T x N queries, masked min).
//
// Mapping on gfx950 (wave64, VALU-bound):
//   one lane = one pose (rollout r, horizon h); the footprint is rotated into
//   the lane's frame once per launch (7 registers per polygon edge); every
//   obstacle point is broadcast to all lanes from LDS, so the inner loop is
//   pure per-lane VALU work with no cross-lane traffic, and the min over
//   points is a private running minimum in a register.  Points are split
//   into chunks over blockIdx.y; the per-chunk minima are merged by the
//   consumer (fixed order, hence deterministic).
//   Distances are kept squared and signed, s = sign(d) d^2 (monotone in d),
//   so one square root per pose replaces one per (point, edge).
#include "kernels.hpp"

namespace emppi {

namespace {

__device__ __forceinline__ float clamp01(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }

// One polygon edge against point (dx, dy) in the frame where the edge is
// (X, Y) -> (X + EX, Y + EY): squared point-to-segment distance with the
// clipped projection alpha = clamp(w.e / |e|^2, 0, 1) (SX, SY = e / |e|^2),
// and the ray-casting quantities: "vertex above the point" (wy < 0) and
// "crossing right of the point" (wx < wy * EX / EY, SL = EX / EY).
struct EdgeEval {
    float d2;
    bool above;
    bool right;
};

__device__ __forceinline__ EdgeEval edge_eval(float dx, float dy, float X, float Y, float EX,
                                              float EY, float SX, float SY, float SL) {
    const float wx = dx - X, wy = dy - Y;
    const float t = clamp01(__builtin_fmaf(wy, SY, wx * SX));
    const float rx = __builtin_fmaf(-t, EX, wx);
    const float ry = __builtin_fmaf(-t, EY, wy);
    EdgeEval e;
    e.d2 = __builtin_fmaf(ry, ry, rx * rx);
    e.above = wy < 0.0f;
    e.right = wx < wy * SL;
    return e;
}

// Signed squared distance of one box (centre c, half extents h) to the
// body-frame point (px, py): with a = |p - c| - h, i = max(a_x, a_y) and
// j = max(min(a_x, a_y), 0), sign(d) d^2 = i |i| + j^2, which equals
// |max(a,0)|^2 outside and -(max(a_x,a_y))^2 inside (the box formula).
__device__ __forceinline__ float box_s(float px, float py, float4 b) {
    const float ax = fabsf(px - b.x) - b.z;
    const float ay = fabsf(py - b.y) - b.w;
    const float i = fmaxf(ax, ay);
    const float j = fmaxf(fminf(ax, ay), 0.0f);
    return __builtin_fmaf(j, j, i * fabsf(i));
}

__device__ __forceinline__ float pose_tau(const PoseTime& pt, int g) {
    const int h = (g / pt.div) % pt.mod;
    return static_cast<float>(h + pt.off) * pt.dt;
}

__device__ __forceinline__ float signed_sqrt(float s) {
    return s < 0.0f ? -__fsqrt_rn(-s) : __fsqrt_rn(s);
}

// Stage points [t0, t0 + tn) of the compacted set into LDS.
template <bool MOVING>
__device__ __forceinline__ void stage_points(float* lds, const PointArgs& pts, int t0, int tn) {
    if (MOVING) {
        float4* l4 = reinterpret_cast<float4*>(lds);
        for (int i = threadIdx.x; i < tn; i += blockDim.x)
            l4[i] = make_float4(pts.x[t0 + i], pts.y[t0 + i], pts.vx[t0 + i], pts.vy[t0 + i]);
    } else {
        float2* l2 = reinterpret_cast<float2*>(lds);
        for (int i = threadIdx.x; i < tn; i += blockDim.x)
            l2[i] = make_float2(pts.x[t0 + i], pts.y[t0 + i]);
    }
}

// Point i of the staged tile at time tau, relative to the pose position.
template <bool MOVING>
__device__ __forceinline__ void point_rel(const float* lds, int i, float tau, float qx, float qy,
                                          float& dx, float& dy) {
    if (MOVING) {
        const float4 o = reinterpret_cast<const float4*>(lds)[i];
        dx = __builtin_fmaf(o.z, tau, o.x) - qx;
        dy = __builtin_fmaf(o.w, tau, o.y) - qy;
    } else {
        const float2 o = reinterpret_cast<const float2*>(lds)[i];
        dx = o.x - qx;
        dy = o.y - qy;
    }
}

// ---------------------------------------------------------------- polygon
// BP = padded vertex count (multiple of 4; padding repeats vertex 0, giving
// zero-length edges that never change the min and never straddle).
// The footprint is used in a frame centred at the pose and aligned with the
// planning frame: vertex b becomes R(theta) v_b, and each point enters as
// o - t (its position relative to the pose).  The distance is rotation
// invariant and the crossing parity does not depend on the ray direction, so
// this equals the body-frame evaluation R(theta)^T (o - t) vs v_b.
template <int BP, bool MOVING, bool ARGMIN>
__global__ __launch_bounds__(256) void k_dmin_poly(const float4* __restrict__ poses, int npose,
                                                   PoseTime pt, PointArgs pts, int chunk,
                                                   const float2* __restrict__ verts,
                                                   float* __restrict__ part,
                                                   int* __restrict__ part_idx) {
    extern __shared__ float lds[];
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = g < npose;
    const float4 q = live ? poses[g] : make_float4(0.f, 0.f, 1.f, 0.f);
    const float tau = MOVING ? pose_tau(pt, g) : 0.0f;

    float X[BP], Y[BP], EX[BP], EY[BP], SX[BP], SY[BP], SL[BP];
#pragma unroll
    for (int b = 0; b < BP; ++b) {
        const float2 v = verts[b];
        X[b] = __builtin_fmaf(q.z, v.x, -(q.w * v.y));
        Y[b] = __builtin_fmaf(q.w, v.x, q.z * v.y);
    }
#pragma unroll
    for (int b = 0; b < BP; ++b) {
        const int bn = (b + 1) % BP;
        EX[b] = X[bn] - X[b];
        EY[b] = Y[bn] - Y[b];
        const float l2 = __builtin_fmaf(EX[b], EX[b], EY[b] * EY[b]);
        const float inv = l2 > 0.0f ? 1.0f / l2 : 0.0f;
        SX[b] = EX[b] * inv;
        SY[b] = EY[b] * inv;
        SL[b] = EY[b] != 0.0f ? EX[b] / EY[b] : 0.0f;
    }

    const int nv = *pts.n_valid;
    const int c0 = blockIdx.y * chunk;
    const int c1 = min(c0 + chunk, nv);
    float best = INFINITY;
    int besti = -1;
    for (int t0 = c0; t0 < c1; t0 += DMIN_TILE) {
        const int tn = min(DMIN_TILE, c1 - t0);
        __syncthreads();
        stage_points<MOVING>(lds, pts, t0, tn);
        __syncthreads();
        for (int i = 0; i < tn; ++i) {
            float dx, dy;
            point_rel<MOVING>(lds, i, tau, q.x, q.y, dx, dy);
            EdgeEval e = edge_eval(dx, dy, X[0], Y[0], EX[0], EY[0], SX[0], SY[0], SL[0]);
            float m = e.d2;
            const bool above0 = e.above;
            bool above = e.above, right = e.right, odd = false;
#pragma unroll
            for (int b = 1; b < BP; ++b) {
                e = edge_eval(dx, dy, X[b], Y[b], EX[b], EY[b], SX[b], SY[b], SL[b]);
                m = fminf(m, e.d2);
                odd ^= (above != e.above) & right;
                above = e.above;
                right = e.right;
            }
            odd ^= (above != above0) & right;
            const float s = odd ? -m : m;
            if (ARGMIN) {
                if (s < best) {
                    best = s;
                    besti = t0 + i;
                }
            } else {
                best = fminf(best, s);
            }
        }
    }
    if (live) {
        const size_t o = static_cast<size_t>(blockIdx.y) * npose + g;
        part[o] = best;
        if (ARGMIN) part_idx[o] = besti >= 0 ? pts.idx[besti] : -1;
    }
}

// ---------------------------------------------------------------- rectangles
// RP = padded box count (padding repeats box 0).  Points are rotated into
// the body frame, p = R(theta)^T (o - t), then evaluated against each box.
template <int RP, bool MOVING, bool ARGMIN>
__global__ __launch_bounds__(256) void k_dmin_rect(const float4* __restrict__ poses, int npose,
                                                   PoseTime pt, PointArgs pts, int chunk,
                                                   const float4* __restrict__ rects,
                                                   float* __restrict__ part,
                                                   int* __restrict__ part_idx) {
    extern __shared__ float lds[];
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = g < npose;
    const float4 q = live ? poses[g] : make_float4(0.f, 0.f, 1.f, 0.f);
    const float tau = MOVING ? pose_tau(pt, g) : 0.0f;
    float4 bx[RP];
#pragma unroll
    for (int j = 0; j < RP; ++j) bx[j] = rects[j];

    const int nv = *pts.n_valid;
    const int c0 = blockIdx.y * chunk;
    const int c1 = min(c0 + chunk, nv);
    float best = INFINITY;
    int besti = -1;
    for (int t0 = c0; t0 < c1; t0 += DMIN_TILE) {
        const int tn = min(DMIN_TILE, c1 - t0);
        __syncthreads();
        stage_points<MOVING>(lds, pts, t0, tn);
        __syncthreads();
        for (int i = 0; i < tn; ++i) {
            float dx, dy;
            point_rel<MOVING>(lds, i, tau, q.x, q.y, dx, dy);
            const float px = __builtin_fmaf(q.z, dx, q.w * dy);
            const float py = __builtin_fmaf(q.z, dy, -(q.w * dx));
            float s = box_s(px, py, bx[0]);
#pragma unroll
            for (int j = 1; j < RP; ++j) s = fminf(s, box_s(px, py, bx[j]));
            if (ARGMIN) {
                if (s < best) {
                    best = s;
                    besti = t0 + i;
                }
            } else {
                best = fminf(best, s);
            }
        }
    }
    if (live) {
        const size_t o = static_cast<size_t>(blockIdx.y) * npose + g;
        part[o] = best;
        if (ARGMIN) part_idx[o] = besti >= 0 ? pts.idx[besti] : -1;
    }
}

// Min over chunks (earlier chunk wins ties: lowest point index), then
// d = sign(s) sqrt(|s|).
__global__ void k_dmin_finalize(const float* __restrict__ part, const int* __restrict__ part_idx,
                                int nchunk, int npose, float* __restrict__ d_out,
                                int* __restrict__ idx_out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npose) return;
    float s = part[g];
    int idx = part_idx ? part_idx[g] : -1;
    for (int c = 1; c < nchunk; ++c) {
        const float v = part[static_cast<size_t>(c) * npose + g];
        if (v < s) {
            s = v;
            if (part_idx) idx = part_idx[static_cast<size_t>(c) * npose + g];
        }
    }
    d_out[g] = signed_sqrt(s);
    if (idx_out) idx_out[g] = idx;
}

// ---------------------------------------------------------------- point-wise
// Body-frame query points, one lane each; the footprint table is uniform
// (scalar loads).  tab_a[b] = (x_b, y_b, ex_b, ey_b), tab_b[b] = (ex_b/|e_b|^2,
// ey_b/|e_b|^2, ex_b/ey_b, 0) for the polygon; tab_a[j] = box j for rects.
__global__ __launch_bounds__(256) void k_sdf_poly_points(const float* __restrict__ px,
                                                         const float* __restrict__ py, int n,
                                                         const float4* __restrict__ ta,
                                                         const float4* __restrict__ tb, int B,
                                                         float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = px[i], y = py[i];
    float4 a = ta[0], b = tb[0];
    EdgeEval e = edge_eval(x, y, a.x, a.y, a.z, a.w, b.x, b.y, b.z);
    float m = e.d2;
    const bool above0 = e.above;
    bool above = e.above, right = e.right, odd = false;
    for (int k = 1; k < B; ++k) {
        a = ta[k];
        b = tb[k];
        e = edge_eval(x, y, a.x, a.y, a.z, a.w, b.x, b.y, b.z);
        m = fminf(m, e.d2);
        odd ^= (above != e.above) & right;
        above = e.above;
        right = e.right;
    }
    odd ^= (above != above0) & right;
    const float d = __fsqrt_rn(m);
    out[i] = odd ? -d : d;
}

__global__ __launch_bounds__(256) void k_sdf_rect_points(const float* __restrict__ px,
                                                         const float* __restrict__ py, int n,
                                                         const float4* __restrict__ ta, int R,
                                                         float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = px[i], y = py[i];
    float s = box_s(x, y, ta[0]);
    for (int j = 1; j < R; ++j) s = fminf(s, box_s(x, y, ta[j]));
    out[i] = signed_sqrt(s);
}

// ---------------------------------------------------------------- compaction
// Order-preserving stream compaction of the valid, finite points (one
// workgroup of 1024 lanes sweeps the array; wave ballots give the offsets).
__global__ __launch_bounds__(1024) void k_compact_points(
    const float* __restrict__ x, const float* __restrict__ y, const float* __restrict__ vx,
    const float* __restrict__ vy, const unsigned char* __restrict__ valid, int n,
    float* __restrict__ ox, float* __restrict__ oy, float* __restrict__ ovx,
    float* __restrict__ ovy, int* __restrict__ oidx, int* __restrict__ n_valid) {
    __shared__ int wsum[16];
    const int lane = threadIdx.x & (WAVE - 1), wid = threadIdx.x / WAVE;
    const int nw = blockDim.x / WAVE;
    int base = 0;
    for (int i0 = 0; i0 < n; i0 += blockDim.x) {
        const int i = i0 + threadIdx.x;
        bool ok = false;
        float a = 0.f, b = 0.f, c = 0.f, d = 0.f;
        if (i < n) {
            a = x[i];
            b = y[i];
            ok = isfinite(a) && isfinite(b);
            if (vx) {
                c = vx[i];
                ok = ok && isfinite(c);
            }
            if (vy) {
                d = vy[i];
                ok = ok && isfinite(d);
            }
            if (valid) ok = ok && valid[i] != 0;
        }
        const uint64_t m = __ballot(ok);
        const int pre = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 0) wsum[wid] = __popcll(m);
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < nw; ++w) {
            off += (w < wid) ? wsum[w] : 0;
            tot += wsum[w];
        }
        if (ok) {
            const int o = base + off + pre;
            ox[o] = a;
            oy[o] = b;
            if (ovx) ovx[o] = c;
            if (ovy) ovy[o] = d;
            oidx[o] = i;
        }
        base += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_valid = base;
}

template <int BP, bool MOVING, bool ARGMIN>
hipError_t launch_poly_t(const DminLaunch& L, dim3 grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_dmin_poly<BP, MOVING, ARGMIN>), grid, dim3(L.block), lds, s, L.poses,
                       L.npose, L.pt, L.pts, L.chunk, L.verts, L.part, L.part_idx);
    return hipGetLastError();
}

template <int RP, bool MOVING, bool ARGMIN>
hipError_t launch_rect_t(const DminLaunch& L, dim3 grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_dmin_rect<RP, MOVING, ARGMIN>), grid, dim3(L.block), lds, s, L.poses,
                       L.npose, L.pt, L.pts, L.chunk, L.rects, L.part, L.part_idx);
    return hipGetLastError();
}

template <int P>
hipError_t launch_kind(const DminLaunch& L, dim3 grid, size_t lds, hipStream_t s) {
    const bool mv = L.pts.vx != nullptr;
    if (L.kind == 0) {
        if (mv) return L.argmin ? launch_poly_t<P, true, true>(L, grid, lds, s)
                                : launch_poly_t<P, true, false>(L, grid, lds, s);
        return L.argmin ? launch_poly_t<P, false, true>(L, grid, lds, s)
                        : launch_poly_t<P, false, false>(L, grid, lds, s);
    }
    if (mv) return L.argmin ? launch_rect_t<P, true, true>(L, grid, lds, s)
                            : launch_rect_t<P, true, false>(L, grid, lds, s);
    return L.argmin ? launch_rect_t<P, false, true>(L, grid, lds, s)
                    : launch_rect_t<P, false, false>(L, grid, lds, s);
}

}  // namespace

int dmin_padded_count(int kind, int count) {
    if (kind == 0) return ((count + 3) / 4) * 4 < 4 ? 4 : ((count + 3) / 4) * 4;
    static const int rb[] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
    for (int b : rb)
        if (count <= b) return b;
    return -1;
}

hipError_t launch_dmin(const DminLaunch& L, hipStream_t s) {
    const dim3 grid((L.npose + L.block - 1) / L.block, L.nchunk);
    const size_t lds = static_cast<size_t>(DMIN_TILE) * (L.pts.vx ? 16 : 8);
    if (L.kind == 0) {
        switch (L.padded) {
        case 4: return launch_kind<4>(L, grid, lds, s);
        case 8: return launch_kind<8>(L, grid, lds, s);
        case 12: return launch_kind<12>(L, grid, lds, s);
        case 16: return launch_kind<16>(L, grid, lds, s);
        case 20: return launch_kind<20>(L, grid, lds, s);
        case 24: return launch_kind<24>(L, grid, lds, s);
        case 28: return launch_kind<28>(L, grid, lds, s);
        case 32: return launch_kind<32>(L, grid, lds, s);
        default: return hipErrorInvalidValue;
        }
    }
    switch (L.padded) {
    case 1: return launch_kind<1>(L, grid, lds, s);
    case 2: return launch_kind<2>(L, grid, lds, s);
    case 3: return launch_kind<3>(L, grid, lds, s);
    case 4: return launch_kind<4>(L, grid, lds, s);
    case 6: return launch_kind<6>(L, grid, lds, s);
    case 8: return launch_kind<8>(L, grid, lds, s);
    case 12: return launch_kind<12>(L, grid, lds, s);
    case 16: return launch_kind<16>(L, grid, lds, s);
    case 24: return launch_kind<24>(L, grid, lds, s);
    case 32: return launch_kind<32>(L, grid, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dmin_finalize(const float* part, const int* part_idx, int nchunk, int npose,
                                float* d_out, int* idx_out, hipStream_t s) {
    if (npose <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dmin_finalize, dim3((npose + 255) / 256), dim3(256), 0, s, part, part_idx,
                       nchunk, npose, d_out, idx_out);
    return hipGetLastError();
}

hipError_t launch_sdf_points(int kind, const float* px, const float* py, int n,
                             const float4* tab_a, const float4* tab_b, int count, float* out,
                             hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const dim3 grid((n + 255) / 256);
    if (kind == 0)
        hipLaunchKernelGGL(k_sdf_poly_points, grid, dim3(256), 0, s, px, py, n, tab_a, tab_b,
                           count, out);
    else
        hipLaunchKernelGGL(k_sdf_rect_points, grid, dim3(256), 0, s, px, py, n, tab_a, count, out);
    return hipGetLastError();
}

hipError_t launch_compact_points(const float* x, const float* y, const float* vx, const float* vy,
                                 const unsigned char* valid, int n, float* ox, float* oy,
                                 float* ovx, float* ovy, int* oidx, int* n_valid, hipStream_t s) {
    hipLaunchKernelGGL(k_compact_points, dim3(1), dim3(1024), 0, s, x, y, vx, vy, valid, n, ox, oy,
                       ovx, ovy, oidx, n_valid);
    return hipGetLastError();
}

}  // namespace emppi
