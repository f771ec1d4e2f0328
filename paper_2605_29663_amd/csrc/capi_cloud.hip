// C ABI of the point-cloud pre-processing pass (declared in
// include/exact_mppi.h): argument checks, the context-owned workspace and
// the launch sequence of kernels_cloud.hip.
#include <cmath>
#include <cstring>

#include "cloud.hpp"
#include "ctx.hpp"

using namespace emppi;
using namespace emppi_host;

static_assert(MPPI_MAX_CLOUD == CLOUD_MAX_POINTS, "cloud capacity of the C ABI");

extern "C" {

int cloud_downsample(mppi_ctx ctx, const float* dxyz, int m, const float center[2],
                     const mppi_cloud_params* cp, float* dx, float* dy, unsigned char* dvalid,
                     int* n_kept) {
    if (!ctx) return MPPI_E_ARG;
    if (!cp || !center) return fail(ctx, MPPI_E_ARG, "cloud: NULL parameters");
    if (m < 0 || m > MPPI_MAX_CLOUD) return fail(ctx, MPPI_E_ARG, "cloud: m=%d outside [0, %d]", m, MPPI_MAX_CLOUD);
    if (cp->n_out < 0 || cp->n_out > MPPI_MAX_CLOUD)
        return fail(ctx, MPPI_E_ARG, "cloud: n_out=%d outside [0, %d]", cp->n_out, MPPI_MAX_CLOUD);
    if (m > 0 && !dxyz) return fail(ctx, MPPI_E_ARG, "cloud: NULL input");
    if (cp->n_out > 0 && (!dx || !dy || !dvalid)) return fail(ctx, MPPI_E_ARG, "cloud: NULL output");
    const float vals[] = {cp->z_min, cp->z_max, cp->r_max, cp->voxel, center[0], center[1]};
    for (float v : vals)
        if (!std::isfinite(v)) return fail(ctx, MPPI_E_ARG, "cloud: non-finite parameter");
    if (!(cp->voxel > 0.0f) || !(cp->r_max > 0.0f) || !(cp->z_min <= cp->z_max))
        return fail(ctx, MPPI_E_ARG, "cloud: need voxel > 0, r_max > 0, z_min <= z_max");
    const double reach = std::max(std::fabs(static_cast<double>(center[0])),
                                  std::fabs(static_cast<double>(center[1]))) + cp->r_max;
    if (reach / cp->voxel >= static_cast<double>(1 << 29))
        return fail(ctx, MPPI_E_ARG, "cloud: voxel too small for the range (voxel index >= 2^29)");
    DeviceGuard g(ctx->device);
    int cap = 256;
    while (cap < 2 * m) cap <<= 1;
    const size_t M = static_cast<size_t>(std::max(m, 1));
    HIP_TRY(ctx, ctx->cloud_keys.ensure(sizeof(unsigned long long) * cap));
    HIP_TRY(ctx, ctx->cloud_first.ensure(sizeof(int) * cap));
    HIP_TRY(ctx, ctx->cloud_cell.ensure(sizeof(unsigned long long) * M));
    HIP_TRY(ctx, ctx->cloud_r2.ensure(sizeof(uint32_t) * M));
    HIP_TRY(ctx, ctx->cloud_misc.ensure(sizeof(int) * (2 * CLOUD_SCAN_BLOCK + 4 * 256 + 8 + 1)));
    CloudArgs a{};
    a.xyz = dxyz;
    a.m = m;
    a.cx = center[0];
    a.cy = center[1];
    a.z_min = cp->z_min;
    a.z_max = cp->z_max;
    a.rmax2 = cp->r_max * cp->r_max;
    a.voxel = cp->voxel;
    a.n_out = cp->n_out;
    CloudWork w{};
    w.keys = ctx->cloud_keys.as<unsigned long long>();
    w.first = ctx->cloud_first.as<int>();
    w.cap_mask = cap - 1;
    w.cell = ctx->cloud_cell.as<unsigned long long>();
    w.r2 = ctx->cloud_r2.as<uint32_t>();
    w.block_sums = ctx->cloud_misc.as<int2>();
    w.hist = ctx->cloud_misc.as<int>() + 2 * CLOUD_SCAN_BLOCK;
    w.state = w.hist + 4 * 256;
    int* d_kept = w.state + 8;
    HIP_TRY(ctx, launch_cloud(a, w, dx, dy, dvalid, d_kept, ctx->stream));
    if (n_kept) {
        HIP_TRY(ctx, hipMemcpyAsync(ctx->h_out, d_kept, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        std::memcpy(n_kept, ctx->h_out, sizeof(int));
    }
    return MPPI_OK;
}

}  // extern "C"
