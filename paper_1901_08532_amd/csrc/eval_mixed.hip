// Mixed-precision evaluation of acceleration, jerk and snap (order 2).
//
// The paper offers a cheaper arithmetic beside full double precision
// (Sec. 3 item 6: an extended type of about 48-bit significand, and single
// precision) for devices weak in double. The mixed form here keeps what
// cancellation makes precision-critical in FP64 and moves the bulk of the
// pair arithmetic to FP32:
//   * position and velocity differences are formed in FP64 from FP64
//     predicted states, then rounded to FP32 (relative error 2^-24 of the
//     small difference, not of the large coordinates);
//   * acceleration differences, the reciprocal square root (v_rsq_f32 and
//     one Newton step), alpha, beta and the pair terms are FP32;
//   * the a/j/s sums are FP64: FP32 products are gathered over 8 sources,
//     then added to plain FP64 accumulators (the FP64 rounding, about 1e-16
//     per addition, stays far below the FP32 terms' own).
// The launch structure (LDS tiles of sources, target per lane, source
// slices, separate compensated slice reduction) is the FP64 kernel's.
#include "eval_mixed_body.h"

namespace h6 {
namespace {

using namespace mixedbody;

template <int BLOCK, int IPL, bool SKIPSELF>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(4))) void k_eval_mixed(
    SrcPtrs src, const int32_t *__restrict__ active, int n, int n_act, double eps2, int slice_len,
    OutPtrs out, int64_t slice_stride) {
    mixed_tile_body<BLOCK, IPL, SKIPSELF>(src, active, n, n_act, eps2, slice_len, out, slice_stride,
                                          blockIdx.x, blockIdx.y);
}

template <int TPW, bool SKIPSELF>
__global__ __launch_bounds__(64) void k_eval_small_mixed(SrcPtrs src,
                                                         const int32_t *__restrict__ active, int n,
                                                         int n_act, double eps2, int slice_len,
                                                         OutPtrs out, int64_t slice_stride) {
    mixed_small_body<TPW, SKIPSELF>(src, active, n, n_act, eps2, slice_len, out, slice_stride,
                                    blockIdx.x, blockIdx.y);
}

template <int BLOCK, int IPL>
hipError_t launch_tile(bool skipself, dim3 grid, hipStream_t st, const SrcPtrs &src,
                       const int32_t *active, int n, int n_act, double eps2, int slice_len,
                       const OutPtrs &out, int64_t slice_stride) {
    if (skipself)
        hipLaunchKernelGGL((k_eval_mixed<BLOCK, IPL, true>), grid, dim3(BLOCK), 0, st, src, active,
                           n, n_act, eps2, slice_len, out, slice_stride);
    else
        hipLaunchKernelGGL((k_eval_mixed<BLOCK, IPL, false>), grid, dim3(BLOCK), 0, st, src,
                           active, n, n_act, eps2, slice_len, out, slice_stride);
    return hipGetLastError();
}

}  // namespace

hipError_t dispatch_mixed(const EvalConfig &cfg, bool skipself, dim3 grid, hipStream_t st,
                          const SrcPtrs &src, const int32_t *active, int n, int n_act, double eps2,
                          int slice_len, const OutPtrs &out, int64_t slice_stride) {
    if (cfg.kind == 1) {
#define H6_SMALLM(T)                                                                            \
    if (cfg.ipl == T) {                                                                         \
        if (skipself)                                                                           \
            hipLaunchKernelGGL((k_eval_small_mixed<T, true>), grid, dim3(64), 0, st, src,       \
                               active, n, n_act, eps2, slice_len, out, slice_stride);           \
        else                                                                                    \
            hipLaunchKernelGGL((k_eval_small_mixed<T, false>), grid, dim3(64), 0, st, src,      \
                               active, n, n_act, eps2, slice_len, out, slice_stride);           \
        return hipGetLastError();                                                               \
    }
        H6_SMALLM(1)
        H6_SMALLM(2)
        H6_SMALLM(4)
#undef H6_SMALLM
        return hipErrorInvalidValue;
    }
#define H6_TILEM(B, I)                                                                          \
    if (cfg.block == B && cfg.ipl == I)                                                         \
        return launch_tile<B, I>(skipself, grid, st, src, active, n, n_act, eps2, slice_len, out, \
                                 slice_stride);
    H6_TILEM(64, 1)
    H6_TILEM(128, 1)
    H6_TILEM(256, 1)
    H6_TILEM(64, 2)
    H6_TILEM(128, 2)
    H6_TILEM(256, 2)
#undef H6_TILEM
    return hipErrorInvalidValue;
}

}  // namespace h6
