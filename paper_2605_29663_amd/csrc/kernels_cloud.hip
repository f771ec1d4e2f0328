// Point-cloud pre-processing (Section "Problem Statement": the obstacle set
// is the local point cloud restricted to a height band and downsampled to a
// fixed budget N).  One representative per occupied planar voxel (its
// lowest-index point), the N nearest representatives if there are more, in
// input order, padded with invalid slots.  Every decision is an exact
// integer or single-precision comparison, so the result does not depend on
// thread scheduling.
#include <algorithm>
#include <climits>

#include "cloud.hpp"

namespace emppi {

namespace {

constexpr unsigned long long CELL_NONE = ~0ull;
// key of a point that represents no voxel: above every squared range (the
// ranges are finite non-negative floats, whose bits stay below 0x7F800000)
constexpr uint32_t KEY_NONE = 0xFFFFFFFFu;
constexpr int CELL_BIAS = 1 << 30;  // voxel coordinates are stored biased, never all ones

// MurmurHash3's 64-bit finaliser (Appleby), used to spread voxel keys over
// the open-addressing table.
__device__ __forceinline__ uint32_t mix64(unsigned long long k) {
    k ^= k >> 33;
    k *= 0xff51afd7ed558ccdull;
    k ^= k >> 33;
    k *= 0xc4ceb9fe1a85ec53ull;
    k ^= k >> 33;
    return static_cast<uint32_t>(k);
}

__global__ void k_cloud_init(CloudWork w) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s <= w.cap_mask) {
        w.keys[s] = CELL_NONE;
        w.first[s] = INT_MAX;
    }
    if (s < 4 * 256) w.hist[s] = 0;
    if (s < 8) w.state[s] = 0;
}

// Height band, range and finiteness test; voxel insertion (the slot keeps
// the minimum index of its points); cell[i] = the point's slot, or CELL_NONE.
__global__ void k_cloud_insert(CloudArgs a, CloudWork w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.m) return;
    const float x = a.xyz[3 * i], y = a.xyz[3 * i + 1], z = a.xyz[3 * i + 2];
    const float dx = x - a.cx, dy = y - a.cy;
    const float r2 = dx * dx + dy * dy;
    const bool ok = isfinite(x) && isfinite(y) && isfinite(z) && z >= a.z_min && z <= a.z_max &&
                    r2 <= a.rmax2;
    w.r2[i] = __float_as_uint(r2);
    unsigned long long key = CELL_NONE;
    if (ok) {
        const int ix = static_cast<int>(floorf(x / a.voxel));
        const int iy = static_cast<int>(floorf(y / a.voxel));
        key = (static_cast<unsigned long long>(static_cast<uint32_t>(ix + CELL_BIAS)) << 32) |
              static_cast<uint32_t>(iy + CELL_BIAS);
        uint32_t slot = mix64(key) & static_cast<uint32_t>(w.cap_mask);
        // the table holds at least twice as many slots as points: a free
        // slot is always reached.  A slot's key is set once and its index
        // only decreases, so a plain (relaxed) read that already shows this
        // key, another key, or an index below i is final, and the atomics
        // run only when the read leaves the outcome open (most points share
        // their voxel with many others)
        for (;;) {
            unsigned long long cur =
                __hip_atomic_load(&w.keys[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cur == CELL_NONE) cur = atomicCAS(&w.keys[slot], CELL_NONE, key);
            if (cur == CELL_NONE || cur == key) {
                if (__hip_atomic_load(&w.first[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > i)
                    atomicMin(&w.first[slot], i);
                break;
            }
            slot = (slot + 1) & static_cast<uint32_t>(w.cap_mask);
        }
        w.cell[i] = slot;
    } else {
        w.cell[i] = CELL_NONE;
    }
}

// The radix-select state (MSB first, 8 bits per pass) towards the need-th
// smallest squared-range key of the representatives, need starting at
// min(representatives, n_out), after `passes` passes: the key prefix, its
// mask and how many keys are still to be taken among those that match the
// prefix.  Pass q takes the first bin b of its histogram whose cumulative
// count reaches need, appends b to the prefix and lowers need by the count
// before b.  Every workgroup that needs the state derives it from the
// histograms of the earlier passes (the same integers, so the same state)
// instead of a separate single-thread launch per pass.  Called by all 64
// lanes of one wave; every lane returns the state.
struct CloudSelect {
    uint32_t prefix, mask;
    int need;
};

__device__ CloudSelect cloud_select(const CloudWork& w, int n_out, int passes) {
    const int lane = static_cast<int>(threadIdx.x) & 63;
    int c[4][4];  // [pass][bin 4 lane + k]: every histogram read at once
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int k = 0; k < 4; ++k) c[q][k] = q < passes ? w.hist[q * 256 + 4 * lane + k] : 0;
    CloudSelect S{0u, 0u, min(w.state[0], n_out)};
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        if (q >= passes || S.need <= 0) break;
        const int ls = c[q][0] + c[q][1] + c[q][2] + c[q][3];
        int incl = ls;
        for (int o = 1; o < 64; o <<= 1) {
            const int t = __shfl_up(incl, o);
            if (lane >= o) incl += t;
        }
        const unsigned long long hit = __ballot(incl >= S.need);
        if (hit == 0) break;  // not reached: the bins of pass q hold >= need keys
        const int L = __ffsll(static_cast<long long>(hit)) - 1;
        int cum = __shfl(incl - ls, L);
        int b = -1, before = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int ck = __shfl(c[q][k], L);
            if (b < 0 && cum + ck >= S.need) {
                b = 4 * L + k;
                before = cum;
            }
            cum += ck;
        }
        const int shift = 24 - 8 * q;
        S.prefix |= static_cast<uint32_t>(b) << shift;
        S.mask |= 255u << shift;
        S.need -= before;
    }
    return S;
}

// Histogram (into hist[pass]) of the next 8 bits of the squared-range keys of
// the representatives that match the prefix the earlier passes decided.
// Pass 0 first decides which points represent their voxel (the lowest index
// of the slot), counts them into state[0], histograms all of them (its
// prefix is empty) and sets the key of every other point to KEY_NONE, above
// any squared range, so that later passes and the selection read one word
// per point.
__global__ __launch_bounds__(256) void k_cloud_hist(int m, CloudWork w, int pass, int n_out) {
    __shared__ int h[256];
    __shared__ uint32_t s_prefix, s_mask;
    __shared__ int s_need;
    __shared__ int cnt;
    h[threadIdx.x] = 0;
    if (pass == 0) {
        if (threadIdx.x == 0) cnt = 0;
        __syncthreads();
        int c = 0;
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
            const unsigned long long slot = w.cell[i];
            const bool f = slot != CELL_NONE && w.first[slot] == i;
            if (f) {
                ++c;
                atomicAdd(&h[w.r2[i] >> 24], 1);
            } else {
                w.r2[i] = KEY_NONE;
            }
        }
        if (c) atomicAdd(&cnt, c);
        __syncthreads();
        if (threadIdx.x == 0 && cnt) atomicAdd(&w.state[0], cnt);
        if (h[threadIdx.x]) atomicAdd(&w.hist[threadIdx.x], h[threadIdx.x]);
        return;
    }
    if (threadIdx.x < 64) {
        const CloudSelect S = cloud_select(w, n_out, pass);
        if (threadIdx.x == 0) {
            s_prefix = S.prefix;
            s_mask = S.mask;
            s_need = S.need;
        }
    }
    __syncthreads();
    const uint32_t prefix = s_prefix, mask = s_mask;
    const int shift = 24 - 8 * pass;
    if (s_need > 0)
        for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
            const uint32_t u = w.r2[i];  // KEY_NONE never matches a prefix of a range key
            if ((u & mask) == prefix) atomicAdd(&h[(u >> shift) & 255u], 1);
        }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&w.hist[pass * 256 + threadIdx.x], h[threadIdx.x]);
}

// Exclusive prefix sums of (below, tie) count pairs over one workgroup of
// CLOUD_SCAN_BLOCK threads (every thread must call it); returns the
// workgroup's totals.
__device__ int2 block_scan2(int2 v, int2& excl) {
    __shared__ int2 wsum[CLOUD_SCAN_BLOCK / 64];
    __shared__ int2 total;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int sx = v.x, sy = v.y;
    for (int o = 1; o < 64; o <<= 1) {
        const int tx = __shfl_up(sx, o), ty = __shfl_up(sy, o);
        if (lane >= o) {
            sx += tx;
            sy += ty;
        }
    }
    if (lane == 63) wsum[wid] = make_int2(sx, sy);
    __syncthreads();
    if (threadIdx.x == 0) {
        int ax = 0, ay = 0;
        for (int k = 0; k < CLOUD_SCAN_BLOCK / 64; ++k) {
            const int2 t = wsum[k];
            wsum[k] = make_int2(ax, ay);
            ax += t.x;
            ay += t.y;
        }
        total = make_int2(ax, ay);
    }
    __syncthreads();
    excl = make_int2(wsum[wid].x + sx - v.x, wsum[wid].y + sy - v.y);
    return total;
}

// Selection, level 1: the final state (threshold key t = the prefix after 4
// passes, need) and, per point, below = representative with key < t and tie
// = representative with key == t (both 0 when nothing is to be taken);
// exclusive sums of both within each block of CLOUD_SCAN_BLOCK points.
// Workgroup 0 records t and need in state[2], state[1].
__global__ __launch_bounds__(CLOUD_SCAN_BLOCK) void k_cloud_scan1(int m, CloudWork w, int n_out,
                                                                  int2* __restrict__ excl) {
    __shared__ uint32_t s_t;
    __shared__ int s_need;
    if (threadIdx.x < 64) {
        const CloudSelect S = cloud_select(w, n_out, 4);
        if (threadIdx.x == 0) {
            s_t = S.prefix;
            s_need = S.need;
            if (blockIdx.x == 0) {
                w.state[1] = S.need;
                w.state[2] = static_cast<int>(S.prefix);
            }
        }
    }
    __syncthreads();
    const int i = blockIdx.x * CLOUD_SCAN_BLOCK + threadIdx.x;
    int2 v = make_int2(0, 0);
    if (i < m && s_need > 0) {
        const uint32_t u = w.r2[i];  // KEY_NONE (not a representative) is above t
        v = make_int2(u < s_t ? 1 : 0, u == s_t ? 1 : 0);
    }
    int2 e;
    const int2 tot = block_scan2(v, e);
    if (i < m) excl[i] = e;
    if (threadIdx.x == 0) w.block_sums[blockIdx.x] = tot;
}

// Level 2 (one workgroup): exclusive sums of the block totals; the kept count
// = representatives below t + min(ties, need) goes to state[5].
__global__ __launch_bounds__(CLOUD_SCAN_BLOCK) void k_cloud_scan2(int nb, CloudWork w) {
    const int2 v = static_cast<int>(threadIdx.x) < nb ? w.block_sums[threadIdx.x] : make_int2(0, 0);
    int2 e;
    const int2 tot = block_scan2(v, e);
    if (static_cast<int>(threadIdx.x) < nb) w.block_sums[threadIdx.x] = e;
    if (threadIdx.x == 0) w.state[5] = tot.x + min(tot.y, max(w.state[1], 0));
}

// Level 3: every representative below t, and the ties of rank < need, go to
// output slot (representatives below t before it) + min(ties before it,
// need), i.e. in input order; slots [kept, n_out) are cleared.  Thread g
// handles point g and output slot g.
__global__ __launch_bounds__(CLOUD_SCAN_BLOCK) void k_cloud_scan3(CloudArgs a, CloudWork w,
                                                                  const int2* __restrict__ excl,
                                                                  float* ox, float* oy,
                                                                  unsigned char* valid,
                                                                  int* n_kept) {
    const int g = blockIdx.x * CLOUD_SCAN_BLOCK + threadIdx.x;
    const int kept = w.state[5], need = w.state[1];
    const uint32_t t = static_cast<uint32_t>(w.state[2]);
    if (g == 0 && n_kept) *n_kept = kept;
    if (g < a.m && need > 0) {
        const uint32_t u = w.r2[g];
        const int2 e = excl[g], b = w.block_sums[blockIdx.x];
        const int below = e.x + b.x, ties = e.y + b.y;
        if (u < t || (u == t && ties < need)) {
            const int pos = below + min(ties, need);
            ox[pos] = a.xyz[3 * g];
            oy[pos] = a.xyz[3 * g + 1];
            valid[pos] = 1;
        }
    }
    if (g < a.n_out && g >= kept) {
        ox[g] = 0.0f;
        oy[g] = 0.0f;
        valid[g] = 0;
    }
}

}  // namespace

// The whole pre-processing pass on stream s (9 launches; 2 when m = 0).
// The (below, tie) prefix sums reuse w.cell (8 bytes per point) once the
// voxel keys are no longer needed.
hipError_t launch_cloud(const CloudArgs& a, const CloudWork& w, float* ox, float* oy,
                        unsigned char* valid, int* n_kept, hipStream_t s) {
    const int cap = w.cap_mask + 1;
    const int n_init = std::max(cap, 4 * 256);  // the table and the four histograms
    hipLaunchKernelGGL(k_cloud_init, dim3((n_init + 255) / 256), dim3(256), 0, s, w);
    const int m = a.m;
    int2* excl = reinterpret_cast<int2*>(w.cell);
    if (m > 0) {
        const dim3 g((m + 255) / 256), b(256);
        hipLaunchKernelGGL(k_cloud_insert, g, b, 0, s, a, w);
        const int hist_blocks = static_cast<int>(std::min<long>((m + 255) / 256, 1024));
        for (int pass = 0; pass < 4; ++pass)
            hipLaunchKernelGGL(k_cloud_hist, dim3(hist_blocks), dim3(256), 0, s, m, w, pass, a.n_out);
        const int nb = (m + CLOUD_SCAN_BLOCK - 1) / CLOUD_SCAN_BLOCK;
        hipLaunchKernelGGL(k_cloud_scan1, dim3(nb), dim3(CLOUD_SCAN_BLOCK), 0, s, m, w, a.n_out, excl);
        hipLaunchKernelGGL(k_cloud_scan2, dim3(1), dim3(CLOUD_SCAN_BLOCK), 0, s, nb, w);
    }
    const int n3 = std::max(std::max(m, a.n_out), 1);
    hipLaunchKernelGGL(k_cloud_scan3, dim3((n3 + CLOUD_SCAN_BLOCK - 1) / CLOUD_SCAN_BLOCK),
                       dim3(CLOUD_SCAN_BLOCK), 0, s, a, w, excl, ox, oy, valid, n_kept);
    return hipGetLastError();
}

}  // namespace emppi
