// Internal interface of the point-cloud pre-processing kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace emppi {

constexpr int CLOUD_SCAN_BLOCK = 1024;              // elements per scan block
constexpr int CLOUD_MAX_POINTS = CLOUD_SCAN_BLOCK * CLOUD_SCAN_BLOCK;  // two-level scan

struct CloudArgs {
    const float* xyz;  // m x 3, row-major
    int m;
    float cx, cy;      // robot position (planning frame)
    float z_min, z_max, rmax2, voxel;
    int n_out;
};

// Device workspace of one pre-processing call (sizes in elements).
struct CloudWork {
    unsigned long long* keys;  // cap: voxel hash table keys
    int* first;                // cap: lowest point index per voxel
    int cap_mask;              // cap - 1 (cap a power of two >= 2 m)
    unsigned long long* cell;  // m: table slot of each kept point (~0 if dropped)
    uint32_t* r2;              // m: squared range bits (KEY_NONE once known not a representative)
    int2* block_sums;          // CLOUD_SCAN_BLOCK: (below, tie) sums per scan block
    int* hist;                 // 4 x 256: one histogram per radix-select pass
    int* state;                // 8: representatives, need, threshold, kept
};

hipError_t launch_cloud(const CloudArgs& a, const CloudWork& w, float* ox, float* oy,
                        unsigned char* valid, int* n_kept, hipStream_t s);

}  // namespace emppi
