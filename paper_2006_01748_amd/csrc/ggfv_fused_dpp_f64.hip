// ggfv_fused_dpp_f64.hip -- the FP64 instances of the lane-shift kernels
// (ggfv_fused_dpp.hpp).  They are compiled apart from the FP32 ones because
// the two precisions run fastest under different instruction schedules: the
// FP32 kernels under the ILP strategy, the FP64 kernels, whose late stores need
// the registers that strategy takes, under the default one.

#include "ggfv_fused_dpp.hpp"

namespace ggfv {

int lane_shift_fit_rows_f64(const ggfv_ctx *ctx, int K, int rounds2, bool wide)
{
    return wide ? fit_rows_depth<double, false, 2>(ctx, K, rounds2) : fit_rows_depth<double, false, 1>(ctx, K, rounds2);
}

hipError_t launch_step_fused_dpp_f64(ggfv_ctx *ctx, const void *in, void *out, double dt, int K, bool wide)
{
    return wide ? launch_dpp_depth<double, false, 2>(ctx, in, out, dt, K)
                : launch_dpp_depth<double, false, 1>(ctx, in, out, dt, K);
}

hipError_t launch_step_batch_dpp_f64(const BatchLaunch &b, hipStream_t stream)
{
    return launch_dpp_batch_depth<double, false, 1>(b, stream);
}

}  // namespace ggfv
