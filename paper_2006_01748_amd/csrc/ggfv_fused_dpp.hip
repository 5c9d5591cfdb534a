// ggfv_fused_dpp.hip -- the FP32 instances of the lane-shift kernels
// (ggfv_fused_dpp.hpp, compiled with the ILP instruction schedule) and the
// entry points that pick a kernel by precision, width and depth; the FP64
// instances are in ggfv_fused_dpp_f64.hip.

#include "ggfv_fused_dpp.hpp"

namespace ggfv {

// lane_shift 1: 8 bytes of columns per lane (one FP64 or two FP32 columns);
// lane_shift 2 (wide lanes): 16 bytes (two FP64 or four FP32 columns), which
// halves the lane shifts, edge selects and halo columns per cell at twice the
// registers.  The compensated state keeps 8 bytes per lane.
int lane_shift_fit_rows(const ggfv_ctx *ctx, int K, int rounds2)
{
    const bool wide = ctx->lane_shift == 2;
    if (ctx->dtype == GGFV_F64) return lane_shift_fit_rows_f64(ctx, K, rounds2, wide);
    if (ctx->dtype == GGFV_F32C) return fit_rows_depth<float, true, 2>(ctx, K, rounds2);
    return wide ? fit_rows_depth<float, false, 4>(ctx, K, rounds2) : fit_rows_depth<float, false, 2>(ctx, K, rounds2);
}

hipError_t launch_step_fused_dpp(ggfv_ctx *ctx, const void *in, void *out, double dt, int K)
{
    const bool wide = ctx->lane_shift == 2;
    switch (ctx->dtype) {
    case GGFV_F64: return launch_step_fused_dpp_f64(ctx, in, out, dt, K, wide);
    case GGFV_F32:
        return wide ? launch_dpp_depth<float, false, 4>(ctx, in, out, dt, K)
                    : launch_dpp_depth<float, false, 2>(ctx, in, out, dt, K);
    case GGFV_F32C: return launch_dpp_depth<float, true, 2>(ctx, in, out, dt, K);
    default: return hipErrorInvalidValue;
    }
}

int lane_shift_columns_per_group(int dtype, int K)
{
    const int cpl = dtype == GGFV_F64 ? 1 : 2;
    const int h = (K + cpl - 1) / cpl * cpl;
    return kWave * cpl - 2 * h;
}

hipError_t launch_step_batch_dpp(const BatchLaunch &b, hipStream_t stream)
{
    if (b.items <= 0) return hipSuccess;
    switch (b.dtype) {
    case GGFV_F64: return launch_step_batch_dpp_f64(b, stream);
    case GGFV_F32: return launch_dpp_batch_depth<float, false, 2>(b, stream);
    case GGFV_F32C: return launch_dpp_batch_depth<float, true, 2>(b, stream);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace ggfv
