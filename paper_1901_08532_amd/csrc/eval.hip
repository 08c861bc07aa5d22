// Evaluation of softened acceleration, jerk, snap (and, at start-up,
// crackle) on a set of target particles from all source particles.
//
// The stage and its kernel steps follow the paper (Sec. 3, item 4): sources
// are staged tile by tile through on-chip local memory (LDS here), each
// thread keeps its target's partial sums in registers across tiles, the
// self term is excluded, and the sums are written to global memory at the
// end. The pair terms are the time derivatives of the softened Newtonian
// acceleration of the 6th-order Hermite scheme the paper cites.
//
// gfx950 design:
//   * one target per lane (or two: IPL = 2), wave64; the source record of a
//     tile entry is read by all lanes at one LDS address (broadcast), five
//     128-bit reads per source;
//   * grid = (target blocks) x (source slices): the sum over sources is
//     split across workgroups so that even a few hundred targets fill 256
//     CUs; the slices are combined by a separate compensated reduction;
//   * FP64 throughout; reciprocal square root from the hardware estimate
//     (v_rsq_f64) refined by one Newton step;
//   * per tile the register sums are flushed into a compensated (hi, lo)
//     pair, so rounding grows with the number of tiles, not sources;
//   * no floating-point atomics: results are bitwise reproducible for a
//     given launch shape.
#include <algorithm>
#include <climits>

#include "eval_body.h"

namespace h6 {
namespace {

using namespace evalbody;

template <int ORDER, int BLOCK, int IPL, bool SKIPSELF>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(IPL == 1 ? 4 : 2))) void k_eval_f64(
    SrcPtrs src, const int32_t *__restrict__ active, int n, int n_act, double eps2, int slice_len,
    OutPtrs out, int64_t slice_stride) {
    eval_tile_body<ORDER, BLOCK, IPL, SKIPSELF>(src, active, n, n_act, eps2, slice_len, out,
                                                slice_stride, blockIdx.x, blockIdx.y);
}

// Slice reduction, few slices: one thread per (component, target), a
// Neumaier sum over the slices with all loads issued up front.
__global__ __launch_bounds__(256) void k_reduce_slices(const double *__restrict__ partial,
                                                       int64_t ld, int n_split, int ncomp, int out0,
                                                       int n_act, OutPtrs out, unsigned acc_mask) {
    const int64_t total = (int64_t)ncomp * n_act;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(idx / n_act);
        const int k = (int)(idx - (int64_t)c * n_act);
        double s = 0.0, comp = 0.0;
        for (int s0 = 0; s0 < n_split; s0 += 8) {
            double x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                x[u] = s0 + u < n_split ? partial[((int64_t)(s0 + u) * ncomp + c) * ld + k] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const double t = s + x[u];
                comp += fabs(s) >= fabs(x[u]) ? (s - t) + x[u] : (x[u] - t) + s;
                s = t;
            }
        }
        double *dst = &out.p[out0 + c][k];
        *dst = ((acc_mask >> c) & 1u) ? *dst + (s + comp) : s + comp;
    }
}

// Slice reduction, many slices: one wave per (component, target). Each lane
// sums every 64th slice (Neumaier), then a fixed butterfly of compensated
// merges combines the lanes, so the result does not depend on timing.
__global__ __launch_bounds__(256) void k_reduce_slices_wave(const double *__restrict__ partial,
                                                            int64_t ld, int n_split, int ncomp,
                                                            int out0, int n_act, OutPtrs out,
                                                            unsigned acc_mask) {
    const int lane = threadIdx.x & 63;
    const int64_t total = (int64_t)ncomp * n_act;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t idx = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); idx < total;
         idx += waves) {
        const int c = (int)(idx / n_act);
        const int k = (int)(idx - (int64_t)c * n_act);
        double s = 0.0, comp = 0.0;
        for (int sl = lane; sl < n_split; sl += 64) {
            const double x = partial[((int64_t)sl * ncomp + c) * ld + k];
            const double t = s + x;
            comp += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
            s = t;
        }
        wave_comp_sum(s, comp);
        if (lane == 0) {
            double *dst = &out.p[out0 + c][k];
            *dst = ((acc_mask >> c) & 1u) ? *dst + (s + comp) : s + comp;
        }
    }
}

template <int TPW, bool SKIPSELF>
__global__ __launch_bounds__(64) void k_eval_small(SrcPtrs src, const int32_t *__restrict__ active,
                                                    int n, int n_act, double eps2, int slice_len,
                                                    OutPtrs out, int64_t slice_stride) {
    eval_small_body<TPW, SKIPSELF>(src, active, n, n_act, eps2, slice_len, out, slice_stride,
                                   blockIdx.x, blockIdx.y);
}

template <int ORDER, int BLOCK, int IPL>
hipError_t dispatch_f64(bool skipself, dim3 grid, hipStream_t st, const SrcPtrs &src,
                        const int32_t *active, int n, int n_act, double eps2, int slice_len,
                        const OutPtrs &out, int64_t slice_stride) {
    if (skipself)
        hipLaunchKernelGGL((k_eval_f64<ORDER, BLOCK, IPL, true>), grid, dim3(BLOCK), 0, st, src,
                           active, n, n_act, eps2, slice_len, out, slice_stride);
    else
        hipLaunchKernelGGL((k_eval_f64<ORDER, BLOCK, IPL, false>), grid, dim3(BLOCK), 0, st, src,
                           active, n, n_act, eps2, slice_len, out, slice_stride);
    return hipGetLastError();
}

template <int ORDER>
hipError_t dispatch_shape(const EvalConfig &cfg, bool skipself, dim3 grid, hipStream_t st,
                          const SrcPtrs &src, const int32_t *active, int n, int n_act,
                          double eps2, int slice_len, const OutPtrs &out, int64_t slice_stride) {
#define H6_SHAPE(B, I)                                                                          \
    if (cfg.block == B && cfg.ipl == I)                                                         \
        return dispatch_f64<ORDER, B, I>(skipself, grid, st, src, active, n, n_act, eps2,     \
                                         slice_len, out, slice_stride);
    if constexpr (ORDER == 2) {
        H6_SHAPE(64, 1)
        H6_SHAPE(128, 1)
        H6_SHAPE(256, 1)
        H6_SHAPE(64, 2)
        H6_SHAPE(128, 2)
        H6_SHAPE(256, 2)
    } else {
        H6_SHAPE(256, 1)
    }
#undef H6_SHAPE
    return hipErrorInvalidValue;
}

int ceil_div(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

hipError_t dispatch_small(int tpw, bool skipself, dim3 grid, hipStream_t st, const SrcPtrs &src,
                          const int32_t *active, int n, int n_act, double eps2, int slice_len,
                          const OutPtrs &out, int64_t slice_stride) {
#define H6_SMALL(T)                                                                            \
    if (tpw == T) {                                                                            \
        if (skipself)                                                                          \
            hipLaunchKernelGGL((k_eval_small<T, true>), grid, dim3(64), 0, st, src, active, n, \
                               n_act, eps2, slice_len, out, slice_stride);                     \
        else                                                                                   \
            hipLaunchKernelGGL((k_eval_small<T, false>), grid, dim3(64), 0, st, src, active, n,\
                               n_act, eps2, slice_len, out, slice_stride);                     \
        return hipGetLastError();                                                              \
    }
    H6_SMALL(1)
    H6_SMALL(2)
    H6_SMALL(4)
#undef H6_SMALL
    return hipErrorInvalidValue;
}

// Above this many slices the reduction gives each output a whole wave.
constexpr int kWaveReduceMinSplit = 24;
// Active sets up to this size use the source-parallel kernel by default.
constexpr int kDefaultSmallMax = 32;
// Waves a launch aims to put in flight (256 CUs x 4 SIMDs x 2).
constexpr int kTargetWaves = 2048;
// Shortest source slice of the source-parallel kernel (4 sources per lane).
constexpr int kSmallMinSlice = 256;

}  // namespace

// Number of source slices for a target-parallel kernel of `block` threads
// per workgroup whose register footprint allows `waves_per_simd` waves on a
// SIMD. A launch of W workgroups runs in rounds of the resident ones (CUs x
// waves per SIMD x 4 SIMDs / waves per workgroup), so it takes about
// ceil(W / resident) x (slice length + per-workgroup overhead); pick the
// slice count minimising that (fewest slices on ties, to keep the
// reduction small), with at least four tiles per slice.
int balanced_split(h6_ctx ctx, int waves_per_simd, int block, int n, int blocks_i) {
    const int wg_per_cu = std::max(1, waves_per_simd * 4 / (block / 64));
    const int64_t resident = (int64_t)ctx->n_cu * wg_per_cu;
    const int max_split = std::max(1, ceil_div(n, 4 * block));
    const int64_t overhead = 2 * block;  // target loads, partial stores, reduction share
    int best = 1;
    int64_t best_cost = INT64_MAX;
    int last_eff = -1;
    for (int sp = 1; sp <= max_split; ++sp) {
        const int slice = ceil_div(ceil_div(n, sp), block) * block;
        const int eff = ceil_div(n, slice);
        if (eff == last_eff) continue;
        last_eff = eff;
        const int64_t w = (int64_t)blocks_i * eff;
        const int64_t rounds = (w + resident - 1) / resident;
        const int64_t cost = rounds * (slice + overhead);
        if (cost < best_cost) {
            best_cost = cost;
            best = eff;
        }
    }
    return best;
}

EvalConfig choose_eval_config(h6_ctx ctx, int order, int precision, int n, int n_act) {
    EvalConfig cfg;
    if (order == 2 && (precision == H6_EX || precision == H6_SP)) {
        cfg.kind = 0;
        cfg.block = kExtBlock;
        cfg.ipl = 1;
        // slices down to one tile: a double-single pair costs ~20x an FP64
        // one, so even small active sets need many workgroups
        const int blocks_i = ceil_div(n_act, kExtBlock);
        int split = std::max(1, ceil_div(4 * ctx->n_cu, blocks_i));
        split = std::min(split, ceil_div(n, kExtBlock));
        const int64_t cap_split = ctx->partial_cap / ((int64_t)9 * n_act);
        if (split > cap_split) split = (int)(cap_split < 1 ? 1 : cap_split);
        cfg.n_split = split < 1 ? 1 : split;
        return cfg;
    }
    const int small_max = ctx->cfg_small >= 0 ? ctx->cfg_small : kDefaultSmallMax;
    if (order == 2 && n_act <= small_max) {
        // source-parallel kernel: one wave per TPW targets
        cfg.kind = 1;
        cfg.block = 64;
        cfg.ipl = ctx->cfg_ipl ? ctx->cfg_ipl : (n_act <= 4 ? 1 : 2);
        const int waves_i = ceil_div(n_act, cfg.ipl);
        int split = ceil_div(kTargetWaves, waves_i);
        const int max_split = ceil_div(n, kSmallMinSlice);
        if (split > max_split) split = max_split;
        if (ctx->cfg_split) split = ctx->cfg_split < ceil_div(n, 64) ? ctx->cfg_split : ceil_div(n, 64);
        const int64_t cap_split = ctx->partial_cap / ((int64_t)9 * n_act);
        if (split > cap_split) split = (int)cap_split;
        cfg.n_split = split < 1 ? 1 : split;
        return cfg;
    }
    cfg.kind = 0;
    if (order != 2) {
        cfg.block = 256;
        cfg.ipl = 1;
    } else {
        // measured on gfx950 at N = 65536: one target per lane in 64-thread
        // workgroups up to 512 targets, two per lane beyond
        cfg.block = ctx->cfg_block ? ctx->cfg_block : (n_act <= 16384 ? 64 : 256);
        cfg.ipl = ctx->cfg_ipl ? (ctx->cfg_ipl > 2 ? 2 : ctx->cfg_ipl) : (n_act <= 512 ? 1 : 2);
    }
    const int per_block = cfg.block * cfg.ipl;
    const int blocks_i = ceil_div(n_act, per_block);
    int split;
    if (ctx->cfg_split && order == 2) {
        split = ctx->cfg_split;
    } else {
        // measured footprints on gfx950: order 2 with one target per lane
        // <= 128 VGPRs (4 waves per SIMD), two per lane <= 256 (2 waves),
        // except the mixed form's (FP32 pair terms, <= 128: 4 waves, and
        // slices enough to fill them, 8% faster at N = 262144); start-up
        // passes <= 128
        const int waves_per_simd =
            (order == 2 && cfg.ipl == 2 && precision != H6_MIXED) ? 2 : 4;
        split = balanced_split(ctx, waves_per_simd, cfg.block, n, blocks_i);
    }
    const int max_by_tiles = ceil_div(n, cfg.block);
    if (split > max_by_tiles) split = max_by_tiles;
    if (split < 1) split = 1;
    // respect the partial-sum capacity
    const int ncomp = order == 2 ? 9 : 6;
    const int64_t cap_split = ctx->partial_cap / ((int64_t)ncomp * (n_act > 0 ? n_act : 1));
    if (split > 1 && split > cap_split) split = (int)(cap_split < 1 ? 1 : cap_split);
    cfg.n_split = split;
    return cfg;
}

hipError_t launch_eval(h6_ctx ctx, int order, int precision, const SrcPtrs &src, int n,
                       const int32_t *active, int n_act, const OutPtrs &out, EvalConfig *used) {
    if (n_act <= 0) return hipSuccess;
    EvalConfig cfg = choose_eval_config(ctx, order, precision, n, n_act);
    // equal slices, each a whole number of tiles
    int slice_len = ceil_div(n, cfg.n_split);
    slice_len = ceil_div(slice_len, cfg.block) * cfg.block;  // whole tiles (64 for kind 1)
    cfg.n_split = ceil_div(n, slice_len);
    if (used) *used = cfg;

    const int ncomp = order == 2 ? 9 : 6;
    const int out0 = order == 3 ? 6 : 0;
    const int per_block = cfg.block * cfg.ipl;
    dim3 grid(ceil_div(n_act, per_block), cfg.n_split);
    const bool skipself = self_pair_masked(ctx->eps2, precision);

    OutPtrs dst;
    int64_t slice_stride = 0;
    if (cfg.n_split == 1) {
        dst = out;
    } else {
        for (int c = 0; c < kMaxOut; ++c) dst.p[c] = nullptr;
        for (int c = 0; c < ncomp; ++c) dst.p[out0 + c] = ctx->partial + (int64_t)c * n_act;
        slice_stride = (int64_t)ncomp * n_act;
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (ctx->prof) {
        hipError_t pe = prof_begin(ctx, &ev0, &ev1);
        if (pe != hipSuccess) return pe;
    }
    hipError_t e;
    if (order == 2 && (precision == H6_EX || precision == H6_SP)) {
        e = dispatch_ext(precision, skipself, grid, ctx->stream, src, active, n, n_act, ctx->eps2,
                         slice_len, dst, slice_stride);
    } else if (order == 2 && precision == H6_MIXED) {
        dim3 g = cfg.kind == 1 ? dim3(ceil_div(n_act, cfg.ipl), cfg.n_split) : grid;
        e = dispatch_mixed(cfg, skipself, g, ctx->stream, src, active, n, n_act, ctx->eps2,
                           slice_len, dst, slice_stride);
    } else if (cfg.kind == 1) {
        dim3 g(ceil_div(n_act, cfg.ipl), cfg.n_split);
        e = dispatch_small(cfg.ipl, skipself, g, ctx->stream, src, active, n, n_act, ctx->eps2,
                           slice_len, dst, slice_stride);
    } else if (order == 1)
        e = dispatch_shape<1>(cfg, skipself, grid, ctx->stream, src, active, n, n_act, ctx->eps2,
                              slice_len, dst, slice_stride);
    else if (order == 2)
        e = dispatch_shape<2>(cfg, skipself, grid, ctx->stream, src, active, n, n_act, ctx->eps2,
                              slice_len, dst, slice_stride);
    else
        e = dispatch_shape<3>(cfg, skipself, grid, ctx->stream, src, active, n, n_act, ctx->eps2,
                              slice_len, dst, slice_stride);
    if (e == hipSuccess && ctx->prof)
        e = prof_end(ctx, ev0, ev1, order, cfg, precision, n_act, (double)n_act * (double)n);
    if (e != hipSuccess || cfg.n_split == 1) return e;
    return launch_reduce(ctx, cfg.n_split, ncomp, out0, n_act, out, 0u);
}

hipError_t launch_reduce(h6_ctx ctx, int n_split, int ncomp, int out0, int n_act,
                         const OutPtrs &out, unsigned acc_mask) {
    const int64_t total = (int64_t)ncomp * n_act;
    if (n_split >= kWaveReduceMinSplit) {
        int rb = ceil_div(total, 4);
        if (rb > 8192) rb = 8192;
        hipLaunchKernelGGL(k_reduce_slices_wave, dim3(rb), dim3(256), 0, ctx->stream, ctx->partial,
                           (int64_t)n_act, n_split, ncomp, out0, n_act, out, acc_mask);
    } else {
        int rb = ceil_div(total, 256);
        if (rb > 4096) rb = 4096;
        hipLaunchKernelGGL(k_reduce_slices, dim3(rb), dim3(256), 0, ctx->stream, ctx->partial,
                           (int64_t)n_act, n_split, ncomp, out0, n_act, out, acc_mask);
    }
    return hipGetLastError();
}

}  // namespace h6
