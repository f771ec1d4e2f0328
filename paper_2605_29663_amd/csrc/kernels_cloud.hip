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
    if (s < 256) w.hist[s] = 0;
    if (s < 8) w.state[s] = 0;
}

// Height band, range and finiteness test; voxel insertion (the slot keeps
// the minimum index of its points).
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
        // slot is always reached
        for (;;) {
            const unsigned long long prev = atomicCAS(&w.keys[slot], CELL_NONE, key);
            if (prev == CELL_NONE || prev == key) {
                atomicMin(&w.first[slot], i);
                break;
            }
            slot = (slot + 1) & static_cast<uint32_t>(w.cap_mask);
        }
    }
    w.cell[i] = key;
}

// flag[i] = point i represents its voxel; the count goes to state[0].
__global__ void k_cloud_rep(int m, CloudWork w) {
    __shared__ int cnt;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int f = 0;
    if (i < m) {
        const unsigned long long key = w.cell[i];
        if (key != CELL_NONE) {
            uint32_t slot = mix64(key) & static_cast<uint32_t>(w.cap_mask);
            while (w.keys[slot] != key) slot = (slot + 1) & static_cast<uint32_t>(w.cap_mask);
            f = w.first[slot] == i;
        }
        w.flag[i] = f;
    }
    if (f) atomicAdd(&cnt, 1);
    __syncthreads();
    if (threadIdx.x == 0 && cnt) atomicAdd(&w.state[0], cnt);
}

// Histogram of the next 8 bits of the squared-range keys of the
// representatives that match the bits decided so far (state[2], mask state[3]).
__global__ void k_cloud_hist(int m, CloudWork w, int shift) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t prefix = static_cast<uint32_t>(w.state[2]), mask = static_cast<uint32_t>(w.state[3]);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
        const uint32_t u = w.r2[i];
        if (w.flag[i] && (u & mask) == prefix) atomicAdd(&h[(u >> shift) & 255u], 1);
    }
    __syncthreads();
    if (h[threadIdx.x]) atomicAdd(&w.hist[threadIdx.x], h[threadIdx.x]);
}

// One radix-select step (MSB first) towards the need-th smallest key:
// state[1] = how many are still to be taken among the keys that match the
// prefix.  Clears the histogram for the next pass.
__global__ void k_cloud_select(CloudWork w, int shift, int first_pass, int n_out) {
    if (threadIdx.x == 0) {
        if (first_pass) w.state[1] = min(w.state[0], n_out);
        int need = w.state[1];
        if (need > 0) {
            int cum = 0;
            for (int b = 0; b < 256; ++b) {
                const int c = w.hist[b];
                if (cum + c >= need) {
                    w.state[2] = static_cast<int>(static_cast<uint32_t>(w.state[2]) |
                                                  (static_cast<uint32_t>(b) << shift));
                    w.state[3] = static_cast<int>(static_cast<uint32_t>(w.state[3]) |
                                                  (255u << shift));
                    w.state[1] = need - cum;
                    break;
                }
                cum += c;
            }
        }
    }
    __syncthreads();
    w.hist[threadIdx.x] = 0;
}

// tmp = representatives whose key equals the threshold state[2] (ties).
__global__ void k_cloud_ties(int m, CloudWork w, int* tmp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    tmp[i] = w.flag[i] && w.r2[i] == static_cast<uint32_t>(w.state[2]) && w.state[1] > 0;
}

// tmp = selected: below the threshold, or a tie among the state[1] of lowest
// index (excl = rank among the ties).
__global__ void k_cloud_pick(int m, CloudWork w, int* tmp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const uint32_t t = static_cast<uint32_t>(w.state[2]);
    const uint32_t u = w.r2[i];
    const bool take_any = w.state[0] > 0 && w.state[1] > 0;
    tmp[i] = w.flag[i] && take_any && (u < t || (u == t && w.excl[i] < w.state[1]));
}

// Exclusive scan, level 1: per block of CLOUD_SCAN_BLOCK elements.
__global__ __launch_bounds__(CLOUD_SCAN_BLOCK) void k_scan_blocks(const int* __restrict__ in, int m,
                                                                  int* __restrict__ excl,
                                                                  int* __restrict__ block_sums) {
    __shared__ int wsum[CLOUD_SCAN_BLOCK / 64];
    const int i = blockIdx.x * CLOUD_SCAN_BLOCK + threadIdx.x;
    const int v = i < m ? in[i] : 0;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int s = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(s, o);
        if (lane >= o) s += t;
    }
    if (lane == 63) wsum[wid] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int k = 0; k < CLOUD_SCAN_BLOCK / 64; ++k) {
            const int t = wsum[k];
            wsum[k] = acc;
            acc += t;
        }
        block_sums[blockIdx.x] = acc;
    }
    __syncthreads();
    if (i < m) excl[i] = wsum[wid] + s - v;
}

// Level 2: exclusive scan of the block sums (one workgroup); total -> *total.
__global__ __launch_bounds__(CLOUD_SCAN_BLOCK) void k_scan_top(int* __restrict__ block_sums, int nb,
                                                               int* __restrict__ total) {
    __shared__ int wsum[CLOUD_SCAN_BLOCK / 64];
    const int v = threadIdx.x < nb ? block_sums[threadIdx.x] : 0;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int s = v;
    for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(s, o);
        if (lane >= o) s += t;
    }
    if (lane == 63) wsum[wid] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int k = 0; k < CLOUD_SCAN_BLOCK / 64; ++k) {
            const int t = wsum[k];
            wsum[k] = acc;
            acc += t;
        }
        if (total) *total = acc;
    }
    __syncthreads();
    if (threadIdx.x < nb) block_sums[threadIdx.x] = wsum[wid] + s - v;
}

__global__ __launch_bounds__(CLOUD_SCAN_BLOCK) void k_scan_add(int* __restrict__ excl, int m,
                                                               const int* __restrict__ block_sums) {
    const int i = blockIdx.x * CLOUD_SCAN_BLOCK + threadIdx.x;
    if (i < m) excl[i] += block_sums[blockIdx.x];
}

__global__ void k_cloud_scatter(CloudArgs a, CloudWork w, const int* __restrict__ tmp, float* ox,
                                float* oy, unsigned char* valid) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.m || !tmp[i]) return;
    const int pos = w.excl[i];
    ox[pos] = a.xyz[3 * i];
    oy[pos] = a.xyz[3 * i + 1];
    valid[pos] = 1;
}

__global__ void k_cloud_fill(int n_out, CloudWork w, float* ox, float* oy, unsigned char* valid,
                             int* n_kept) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int kept = w.state[5];
    if (j == 0 && n_kept) *n_kept = kept;
    if (j >= n_out || j < kept) return;
    ox[j] = 0.0f;
    oy[j] = 0.0f;
    valid[j] = 0;
}

hipError_t scan(const int* in, int m, CloudWork w, int* total, hipStream_t s) {
    const int nb = (m + CLOUD_SCAN_BLOCK - 1) / CLOUD_SCAN_BLOCK;
    hipLaunchKernelGGL(k_scan_blocks, dim3(nb), dim3(CLOUD_SCAN_BLOCK), 0, s, in, m, w.excl,
                       w.block_sums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(CLOUD_SCAN_BLOCK), 0, s, w.block_sums, nb, total);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(CLOUD_SCAN_BLOCK), 0, s, w.excl, m, w.block_sums);
    return hipGetLastError();
}

}  // namespace

// The whole pre-processing pass on stream s; `tmp` is w.cell reused as an
// int array once the voxel keys are no longer needed (it holds 2 m ints).
hipError_t launch_cloud(const CloudArgs& a, const CloudWork& w, float* ox, float* oy,
                        unsigned char* valid, int* n_kept, hipStream_t s) {
    const int cap = w.cap_mask + 1;
    hipLaunchKernelGGL(k_cloud_init, dim3((cap + 255) / 256), dim3(256), 0, s, w);
    const int m = a.m;
    if (m > 0) {
        const dim3 g((m + 255) / 256), b(256);
        hipLaunchKernelGGL(k_cloud_insert, g, b, 0, s, a, w);
        hipLaunchKernelGGL(k_cloud_rep, g, b, 0, s, m, w);
        const int hist_blocks = static_cast<int>(std::min<long>((m + 255) / 256, 1024));
        for (int pass = 0; pass < 4; ++pass) {
            const int shift = 24 - 8 * pass;
            hipLaunchKernelGGL(k_cloud_hist, dim3(hist_blocks), dim3(256), 0, s, m, w, shift);
            hipLaunchKernelGGL(k_cloud_select, dim3(1), dim3(256), 0, s, w, shift, pass == 0 ? 1 : 0,
                               a.n_out);
        }
        int* tmp = reinterpret_cast<int*>(w.cell);
        hipLaunchKernelGGL(k_cloud_ties, g, b, 0, s, m, w, tmp);
        if (hipError_t e = scan(tmp, m, w, nullptr, s)) return e;
        hipLaunchKernelGGL(k_cloud_pick, g, b, 0, s, m, w, tmp);
        if (hipError_t e = scan(tmp, m, w, w.state + 5, s)) return e;
        hipLaunchKernelGGL(k_cloud_scatter, g, b, 0, s, a, w, tmp, ox, oy, valid);
    }
    const int nf = a.n_out > 0 ? a.n_out : 1;
    hipLaunchKernelGGL(k_cloud_fill, dim3((nf + 255) / 256), dim3(256), 0, s, a.n_out, w, ox, oy,
                       valid, n_kept);
    return hipGetLastError();
}

}  // namespace emppi
