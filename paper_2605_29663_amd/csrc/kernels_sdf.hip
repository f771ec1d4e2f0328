// Single-scene kernels of the fused rollout-frame transform + exact signed
// distance + min over points stage, the point-wise signed-distance kernels,
// and the obstacle-point compaction that implements the validity mask.
// The per-lane work is in sdf_device.hpp (shared with the batched kernel).
#include "sdf_device.hpp"

namespace emppi {

namespace {

// Grid: x over poses (one lane each), y over point chunks of `chunk` points.
// Each chunk's minimum is merged into the pose's key with atomicMin.
// Waves per SIMD the register budget is tuned for (512 VGPRs per lane).
template <int BP>
constexpr int poly_waves() { return BP <= 8 ? 6 : BP <= 16 ? 4 : BP <= 20 ? 3 : 2; }

template <int BP, bool MOVING, bool ARGMIN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(poly_waves<BP>())))
void k_dmin_poly(const float4* __restrict__ poses, int npose,
                                                   PoseTime pt, PointArgs pts, int chunk,
                                                   const float2* __restrict__ verts,
                                                   unsigned int* __restrict__ key,
                                                   unsigned long long* __restrict__ key64) {
    extern __shared__ __align__(16) float lds[];  // point tiles: 8- and 16-byte LDS accesses
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = g < npose;
    const float4 q = live ? poses[g] : make_float4(0.f, 0.f, 1.f, 0.f);
    const float tau = MOVING ? pose_tau(pt, g) : 0.0f;
    const int nv = *pts.n_valid;
    const int c0 = blockIdx.y * chunk;
    const int c1 = min(c0 + chunk, nv);
    float best;
    int besti;
    dmin_poly_range<BP, MOVING, ARGMIN>(q, tau, pts, c0, c1, verts, lds, best, besti);
    if (live) {
        if (ARGMIN) {
            const unsigned int idx = besti >= 0 ? static_cast<unsigned int>(pts.idx[besti]) : 0xFFFFFFFFu;
            atomicMin(&key64[g], (static_cast<unsigned long long>(dkey(best)) << 32) | idx);
        } else {
            atomicMin(&key[g], dkey(best));
        }
    }
}

// Polygons of more than 16 padded vertices: a group of L lanes per pose (a
// pair up to 32 vertices, a quad above), each lane holding HB edges
// (PolyPart); the group's first lane merges the pose's key.  Register
// budget: 4 waves per SIMD for static points (at 16 edges per lane the
// compiler then spills only in the set-up, not in the point loop), 3 for
// moving points (whose point loop would spill at 4).
template <int HB, int L, bool MOVING, bool ARGMIN>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MOVING ? 3 : 4)))
void k_dmin_poly_part(const float4* __restrict__ poses, int npose, PoseTime pt, PointArgs pts,
                      int chunk, const float2* __restrict__ verts, unsigned int* __restrict__ key,
                      unsigned long long* __restrict__ key64) {
    extern __shared__ __align__(16) float lds[];  // point tiles: 8- and 16-byte LDS accesses
    const int g = static_cast<int>((blockIdx.x * blockDim.x + threadIdx.x) / L);
    const bool live = g < npose;
    const float4 q = live ? poses[g] : make_float4(0.f, 0.f, 1.f, 0.f);
    const float tau = MOVING ? pose_tau(pt, g) : 0.0f;
    const int nv = *pts.n_valid;
    const int c0 = blockIdx.y * chunk;
    const int c1 = min(c0 + chunk, nv);
    float best;
    int besti;
    dmin_poly_part_range<HB, L, MOVING, ARGMIN>(q, tau, pts, c0, c1, verts, lds, best, besti);
    if (live && (threadIdx.x & (L - 1)) == 0) {
        if (ARGMIN) {
            const unsigned int idx = besti >= 0 ? static_cast<unsigned int>(pts.idx[besti]) : 0xFFFFFFFFu;
            atomicMin(&key64[g], (static_cast<unsigned long long>(dkey(best)) << 32) | idx);
        } else {
            atomicMin(&key[g], dkey(best));
        }
    }
}

template <int RP, bool MOVING, bool ARGMIN>
__global__ __launch_bounds__(256) void k_dmin_rect(const float4* __restrict__ poses, int npose,
                                                   PoseTime pt, PointArgs pts, int chunk,
                                                   const float4* __restrict__ rects,
                                                   unsigned int* __restrict__ key,
                                                   unsigned long long* __restrict__ key64) {
    extern __shared__ __align__(16) float lds[];  // point tiles: 8- and 16-byte LDS accesses
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = g < npose;
    const float4 q = live ? poses[g] : make_float4(0.f, 0.f, 1.f, 0.f);
    const float tau = MOVING ? pose_tau(pt, g) : 0.0f;
    const int nv = *pts.n_valid;
    const int c0 = blockIdx.y * chunk;
    const int c1 = min(c0 + chunk, nv);
    float best;
    int besti;
    dmin_rect_range<RP, MOVING, ARGMIN>(q, tau, pts, c0, c1, rects, lds, best, besti);
    if (live) {
        if (ARGMIN) {
            const unsigned int idx = besti >= 0 ? static_cast<unsigned int>(pts.idx[besti]) : 0xFFFFFFFFu;
            atomicMin(&key64[g], (static_cast<unsigned long long>(dkey(best)) << 32) | idx);
        } else {
            atomicMin(&key[g], dkey(best));
        }
    }
}

__global__ void k_key_init(unsigned int* __restrict__ key, unsigned long long* __restrict__ key64,
                           int n) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    if (key) key[g] = DKEY_INIT;
    if (key64) key64[g] = DKEY64_INIT;
}

// Keys -> d = sign(s) sqrt(|s|) and the argmin index.
__global__ void k_dmin_finalize(const unsigned int* __restrict__ key,
                                const unsigned long long* __restrict__ key64, int npose,
                                float* __restrict__ d_out, int* __restrict__ idx_out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= npose) return;
    if (key64) {
        const unsigned long long k = key64[g];
        d_out[g] = signed_sqrt(dkey_value(static_cast<unsigned int>(k >> 32)));
        if (idx_out) idx_out[g] = static_cast<int>(static_cast<unsigned int>(k));
    } else {
        d_out[g] = signed_sqrt(dkey_value(key[g]));
        if (idx_out) idx_out[g] = -1;
    }
}

// ---------------------------------------------------------------- point-wise
// Body-frame query points, one lane each; the footprint table is uniform
// (scalar loads).  Polygon: tab_a[b] = (ex, ey, nc, cv) and tab_b[b] = (l,
// y_b, 0, 0) of edge b (EdgeC); rectangle cover: tab_a[j] = box j.
__global__ __launch_bounds__(256) void k_sdf_poly_points(const float* __restrict__ px,
                                                         const float* __restrict__ py, int n,
                                                         const float4* __restrict__ ta,
                                                         const float4* __restrict__ tb, int B,
                                                         float* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = px[i], y = py[i];
    float4 a = ta[0], b = tb[0];
    EdgeEval e = edge_eval(x, y, b.y, a.x, a.y, a.z, a.w, b.x);
    float m = e.d2;
    const bool above0 = e.above;
    bool above = e.above, right = e.right, odd = false;
    for (int k = 1; k < B; ++k) {
        a = ta[k];
        b = tb[k];
        e = edge_eval(x, y, b.y, a.x, a.y, a.z, a.w, b.x);
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
                       L.npose, L.pt, L.pts, L.chunk, L.verts, L.key, L.key64);
    return hipGetLastError();
}

template <int RP, bool MOVING, bool ARGMIN>
hipError_t launch_rect_t(const DminLaunch& L, dim3 grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_dmin_rect<RP, MOVING, ARGMIN>), grid, dim3(L.block), lds, s, L.poses,
                       L.npose, L.pt, L.pts, L.chunk, L.rects, L.key, L.key64);
    return hipGetLastError();
}

template <int HB, int L, bool MOVING, bool ARGMIN>
hipError_t launch_part_t(const DminLaunch& D, dim3 grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_dmin_poly_part<HB, L, MOVING, ARGMIN>), grid, dim3(D.block), lds, s,
                       D.poses, D.npose, D.pt, D.pts, D.chunk, D.verts, D.key, D.key64);
    return hipGetLastError();
}

template <int HB, int L>
hipError_t launch_part(const DminLaunch& D, dim3 grid, size_t lds, hipStream_t s) {
    // L lanes per pose
    const dim3 gl((L * D.npose + D.block - 1) / D.block, grid.y);
    if (D.pts.vx) return D.argmin ? launch_part_t<HB, L, true, true>(D, gl, lds, s)
                                  : launch_part_t<HB, L, true, false>(D, gl, lds, s);
    return D.argmin ? launch_part_t<HB, L, false, true>(D, gl, lds, s)
                    : launch_part_t<HB, L, false, false>(D, gl, lds, s);
}

template <int P>
hipError_t launch_poly(const DminLaunch& L, dim3 grid, size_t lds, hipStream_t s) {
    if constexpr (P > 32) {
        return launch_part<P / 4, 4>(L, grid, lds, s);
    } else if constexpr (P > 16) {
        return launch_part<P / 2, 2>(L, grid, lds, s);
    } else {
        if (L.pts.vx) return L.argmin ? launch_poly_t<P, true, true>(L, grid, lds, s)
                                      : launch_poly_t<P, true, false>(L, grid, lds, s);
        return L.argmin ? launch_poly_t<P, false, true>(L, grid, lds, s)
                        : launch_poly_t<P, false, false>(L, grid, lds, s);
    }
}

template <int P>
hipError_t launch_rect(const DminLaunch& L, dim3 grid, size_t lds, hipStream_t s) {
    if (L.pts.vx) return L.argmin ? launch_rect_t<P, true, true>(L, grid, lds, s)
                                  : launch_rect_t<P, true, false>(L, grid, lds, s);
    return L.argmin ? launch_rect_t<P, false, true>(L, grid, lds, s)
                    : launch_rect_t<P, false, false>(L, grid, lds, s);
}

}  // namespace

int dmin_padded_count(int kind, int count) {
    // polygons: the exact count up to 16 vertices (one lane per pose), even
    // counts up to 32 (a lane pair per pose, half the edges each), multiples
    // of 4 above (a lane quad per pose); padding repeats vertex 0:
    // zero-length edges that change neither the minimum nor the crossing
    // parity
    if (kind == 0) {
        if (count <= 16) return count < 3 ? 3 : count;
        return count <= 32 ? ((count + 1) / 2) * 2 : ((count + 3) / 4) * 4;
    }
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
#define EMPPI_CASE(P) \
    case P: return launch_poly<P>(L, grid, lds, s);
            EMPPI_CASE(3) EMPPI_CASE(4) EMPPI_CASE(5) EMPPI_CASE(6) EMPPI_CASE(7) EMPPI_CASE(8)
            EMPPI_CASE(9) EMPPI_CASE(10) EMPPI_CASE(11) EMPPI_CASE(12) EMPPI_CASE(13)
            EMPPI_CASE(14) EMPPI_CASE(15) EMPPI_CASE(16) EMPPI_CASE(18) EMPPI_CASE(20)
            EMPPI_CASE(22) EMPPI_CASE(24) EMPPI_CASE(26) EMPPI_CASE(28) EMPPI_CASE(30)
            EMPPI_CASE(32) EMPPI_CASE(36) EMPPI_CASE(40) EMPPI_CASE(44) EMPPI_CASE(48)
            EMPPI_CASE(52) EMPPI_CASE(56) EMPPI_CASE(60) EMPPI_CASE(64)
#undef EMPPI_CASE
        default: return hipErrorInvalidValue;
        }
    }
    switch (L.padded) {
    case 1: return launch_rect<1>(L, grid, lds, s);
    case 2: return launch_rect<2>(L, grid, lds, s);
    case 3: return launch_rect<3>(L, grid, lds, s);
    case 4: return launch_rect<4>(L, grid, lds, s);
    case 6: return launch_rect<6>(L, grid, lds, s);
    case 8: return launch_rect<8>(L, grid, lds, s);
    case 12: return launch_rect<12>(L, grid, lds, s);
    case 16: return launch_rect<16>(L, grid, lds, s);
    case 24: return launch_rect<24>(L, grid, lds, s);
    case 32: return launch_rect<32>(L, grid, lds, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_key_init(unsigned int* key, unsigned long long* key64, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_key_init, dim3((n + 255) / 256), dim3(256), 0, s, key, key64, n);
    return hipGetLastError();
}

hipError_t launch_dmin_finalize(const unsigned int* key, const unsigned long long* key64, int npose,
                                float* d_out, int* idx_out, hipStream_t s) {
    if (npose <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_dmin_finalize, dim3((npose + 255) / 256), dim3(256), 0, s, key, key64,
                       npose, d_out, idx_out);
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
