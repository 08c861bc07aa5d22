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
//     (v_rsq_f64) refined by one third-order Newton step;
//   * per tile the register sums are flushed into a compensated (hi, lo)
//     pair, so rounding grows with the number of tiles, not sources;
//   * no floating-point atomics: results are bitwise reproducible for a
//     given launch shape.
#include "h6_internal.h"

namespace h6 {
namespace {

template <int ORDER>
struct Traits;
// ORDER 1: a, j from x, v (start-up pass 1)
template <>
struct Traits<1> {
    static constexpr int NREC = 4;  // double2 per LDS source record
    static constexpr int NACC = 6;
    static constexpr int OUT0 = 0;
};
// ORDER 2: a, j, s from x, v, a (every step)
template <>
struct Traits<2> {
    static constexpr int NREC = 5;
    static constexpr int NACC = 9;
    static constexpr int OUT0 = 0;
};
// ORDER 3: s, c from x, v, a, j (start-up pass 2)
template <>
struct Traits<3> {
    static constexpr int NREC = 7;
    static constexpr int NACC = 6;
    static constexpr int OUT0 = 6;
};

// 1/sqrt(r2): hardware estimate plus one Newton step of third order,
//   e = 1 - r2 y^2,  y <- y (1 + e/2 + 3 e^2/8),
// which takes a relative error d to about (5/2) d^3.
__device__ __forceinline__ double rsqrt_f64(double r2) {
    double y = __builtin_amdgcn_rsq(r2);
    double t = r2 * y;
    double e = fma(-t, y, 1.0);
    double p = fma(e, 0.375, 0.5);
    double ye = y * e;
    return fma(ye, p, y);
}

// hi + lo += x without loss (Knuth's TwoSum on hi, error into lo).
__device__ __forceinline__ void two_sum_into(double &hi, double &lo, double x) {
    double s = hi + x;
    double bp = s - hi;
    double err = (hi - (s - bp)) + (x - bp);
    hi = s;
    lo += err;
}

// Far, massless padding source: contributes exactly zero.
constexpr double kPadPos = 1.0e18;

template <int ORDER, int BLOCK, int IPL, bool SKIPSELF>
__global__ __launch_bounds__(BLOCK) void k_eval_f64(SrcPtrs src, const int32_t *__restrict__ active,
                                                    int n, int n_act, double eps2, int slice_len,
                                                    OutPtrs out, int64_t slice_stride) {
    using T = Traits<ORDER>;
    constexpr int NREC = T::NREC;
    constexpr int NACC = T::NACC;
    __shared__ double2 tile[BLOCK * NREC];
    const int tid = threadIdx.x;

    // ---- targets: predicted state of particle active[k]
    double xi[IPL][3], vi[IPL][3], ai[IPL][3], ji[IPL][3];
    int pid[IPL], kid[IPL];
#pragma unroll
    for (int u = 0; u < IPL; ++u) {
        int k = ((int)blockIdx.x * IPL + u) * BLOCK + tid;
        kid[u] = k;
        int kc = k < n_act ? k : n_act - 1;
        int p = active ? active[kc] : kc;
        pid[u] = p;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xi[u][c] = src.x[c][p];
            vi[u][c] = src.v[c][p];
            ai[u][c] = ORDER >= 2 ? src.a[c][p] : 0.0;
            ji[u][c] = ORDER >= 3 ? src.j[c][p] : 0.0;
        }
    }

    double acc[IPL][NACC], hi[IPL][NACC], lo[IPL][NACC];
#pragma unroll
    for (int u = 0; u < IPL; ++u)
#pragma unroll
        for (int q = 0; q < NACC; ++q) acc[u][q] = hi[u][q] = lo[u][q] = 0.0;

    const int jb = (int)blockIdx.y * slice_len;
    const int je = min(n, jb + slice_len);

    for (int jt = jb; jt < je; jt += BLOCK) {
        __syncthreads();  // previous tile fully consumed
        {
            const int jj = jt + tid;
            double2 *rec = &tile[tid * NREC];
            if (jj < je) {
                rec[0] = make_double2(src.x[0][jj], src.x[1][jj]);
                rec[1] = make_double2(src.x[2][jj], src.m[jj]);
                rec[2] = make_double2(src.v[0][jj], src.v[1][jj]);
                if (ORDER == 1) {
                    rec[3] = make_double2(src.v[2][jj], 0.0);
                } else {
                    rec[3] = make_double2(src.v[2][jj], src.a[0][jj]);
                    rec[4] = make_double2(src.a[1][jj], src.a[2][jj]);
                }
                if (ORDER == 3) {
                    rec[5] = make_double2(src.j[0][jj], src.j[1][jj]);
                    rec[6] = make_double2(src.j[2][jj], 0.0);
                }
            } else {
                rec[0] = make_double2(kPadPos, kPadPos);
                rec[1] = make_double2(kPadPos, 0.0);
#pragma unroll
                for (int q = 2; q < NREC; ++q) rec[q] = make_double2(0.0, 0.0);
            }
        }
        __syncthreads();

#pragma unroll 2
        for (int q = 0; q < BLOCK; ++q) {
            const double2 *rec = &tile[q * NREC];
            const double2 r0 = rec[0], r1 = rec[1], r2v = rec[2], r3 = rec[3];
            const double xj0 = r0.x, xj1 = r0.y, xj2 = r1.x, mj = r1.y;
            const double vj0 = r2v.x, vj1 = r2v.y, vj2 = r3.x;
            double aj0 = 0, aj1 = 0, aj2 = 0, jj0 = 0, jj1 = 0, jj2 = 0;
            if (ORDER >= 2) {
                const double2 r4 = rec[4];
                aj0 = r3.y;
                aj1 = r4.x;
                aj2 = r4.y;
            }
            if (ORDER == 3) {
                const double2 r5 = rec[5], r6 = rec[6];
                jj0 = r5.x;
                jj1 = r5.y;
                jj2 = r6.x;
            }
#pragma unroll
            for (int u = 0; u < IPL; ++u) {
                const double dx = xj0 - xi[u][0], dy = xj1 - xi[u][1], dz = xj2 - xi[u][2];
                const double dvx = vj0 - vi[u][0], dvy = vj1 - vi[u][1], dvz = vj2 - vi[u][2];
                double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
                double m_eff = mj;
                if (SKIPSELF) {
                    const bool self = (jt + q) == pid[u];
                    r2 = self ? 1.0 : r2;
                    m_eff = self ? 0.0 : mj;
                }
                const double rinv = rsqrt_f64(r2);
                const double rinv2 = rinv * rinv;
                const double mr3 = (m_eff * rinv) * rinv2;
                const double rv = fma(dz, dvz, fma(dy, dvy, dx * dvx));
                const double alpha = rv * rinv2;
                const double a3 = 3.0 * alpha;
                // w = v - 3 alpha r, so that J = mr3 w
                const double wx = fma(-a3, dx, dvx), wy = fma(-a3, dy, dvy), wz = fma(-a3, dz, dvz);
                if (ORDER == 1) {
                    acc[u][0] = fma(mr3, dx, acc[u][0]);
                    acc[u][1] = fma(mr3, dy, acc[u][1]);
                    acc[u][2] = fma(mr3, dz, acc[u][2]);
                    acc[u][3] = fma(mr3, wx, acc[u][3]);
                    acc[u][4] = fma(mr3, wy, acc[u][4]);
                    acc[u][5] = fma(mr3, wz, acc[u][5]);
                } else {
                    const double dax = aj0 - ai[u][0], day = aj1 - ai[u][1], daz = aj2 - ai[u][2];
                    // v.v + r.a
                    const double vvra = fma(dz, daz, fma(dy, day, fma(dx, dax,
                                        fma(dvz, dvz, fma(dvy, dvy, dvx * dvx)))));
                    const double beta = fma(alpha, alpha, vvra * rinv2);
                    const double b3 = 3.0 * beta;
                    const double a6 = a3 + a3;
                    // u = a - 6 alpha w - 3 beta r, so that S = mr3 u
                    const double ux = fma(-a6, wx, fma(-b3, dx, dax));
                    const double uy = fma(-a6, wy, fma(-b3, dy, day));
                    const double uz = fma(-a6, wz, fma(-b3, dz, daz));
                    if (ORDER == 2) {
                        acc[u][0] = fma(mr3, dx, acc[u][0]);
                        acc[u][1] = fma(mr3, dy, acc[u][1]);
                        acc[u][2] = fma(mr3, dz, acc[u][2]);
                        acc[u][3] = fma(mr3, wx, acc[u][3]);
                        acc[u][4] = fma(mr3, wy, acc[u][4]);
                        acc[u][5] = fma(mr3, wz, acc[u][5]);
                        acc[u][6] = fma(mr3, ux, acc[u][6]);
                        acc[u][7] = fma(mr3, uy, acc[u][7]);
                        acc[u][8] = fma(mr3, uz, acc[u][8]);
                    } else {
                        const double djx = jj0 - ji[u][0], djy = jj1 - ji[u][1], djz = jj2 - ji[u][2];
                        const double va = fma(dvz, daz, fma(dvy, day, dvx * dax));
                        const double rj = fma(dz, djz, fma(dy, djy, dx * djx));
                        // gamma = (3 v.a + r.j)/R^2 + alpha (3 beta - 4 alpha^2)
                        const double gamma = fma(alpha, fma(-4.0 * alpha, alpha, b3),
                                                 fma(3.0, va, rj) * rinv2);
                        const double a9 = 3.0 * a3, b9 = 3.0 * b3, g3 = 3.0 * gamma;
                        // z = jr - 9 alpha u - 9 beta w - 3 gamma r, so that C = mr3 z
                        const double zx = fma(-a9, ux, fma(-b9, wx, fma(-g3, dx, djx)));
                        const double zy = fma(-a9, uy, fma(-b9, wy, fma(-g3, dy, djy)));
                        const double zz = fma(-a9, uz, fma(-b9, wz, fma(-g3, dz, djz)));
                        acc[u][0] = fma(mr3, ux, acc[u][0]);
                        acc[u][1] = fma(mr3, uy, acc[u][1]);
                        acc[u][2] = fma(mr3, uz, acc[u][2]);
                        acc[u][3] = fma(mr3, zx, acc[u][3]);
                        acc[u][4] = fma(mr3, zy, acc[u][4]);
                        acc[u][5] = fma(mr3, zz, acc[u][5]);
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < IPL; ++u)
#pragma unroll
            for (int q = 0; q < NACC; ++q) {
                two_sum_into(hi[u][q], lo[u][q], acc[u][q]);
                acc[u][q] = 0.0;
            }
    }

    const int64_t soff = (int64_t)blockIdx.y * slice_stride;
#pragma unroll
    for (int u = 0; u < IPL; ++u) {
        if (kid[u] < n_act) {
#pragma unroll
            for (int q = 0; q < NACC; ++q) out.p[T::OUT0 + q][soff + kid[u]] = hi[u][q] + lo[u][q];
        }
    }
}

// Compensated (Neumaier) sum of the per-slice partials of each target.
__global__ __launch_bounds__(256) void k_reduce_slices(const double *__restrict__ partial,
                                                       int64_t ld, int n_split, int ncomp, int out0,
                                                       int n_act, OutPtrs out) {
    const int64_t total = (int64_t)ncomp * n_act;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(idx / n_act);
        const int k = (int)(idx - (int64_t)c * n_act);
        double s = 0.0, comp = 0.0;
        for (int sl = 0; sl < n_split; ++sl) {
            const double x = partial[((int64_t)sl * ncomp + c) * ld + k];
            const double t = s + x;
            comp += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
            s = t;
        }
        out.p[out0 + c][k] = s + comp;
    }
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
    if (ORDER == 2) {
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

}  // namespace

EvalConfig choose_eval_config(h6_ctx ctx, int order, int precision, int n, int n_act) {
    (void)precision;
    EvalConfig cfg;
    if (order != 2) {
        cfg.block = 256;
        cfg.ipl = 1;
    } else {
        cfg.block = ctx->cfg_block ? ctx->cfg_block : (n_act <= 2048 ? 64 : 256);
        cfg.ipl = ctx->cfg_ipl ? ctx->cfg_ipl : 1;
    }
    const int per_block = cfg.block * cfg.ipl;
    const int blocks_i = ceil_div(n_act, per_block);
    int split;
    if (ctx->cfg_split && order == 2) {
        split = ctx->cfg_split;
    } else {
        // aim at about 8 workgroups per CU on 256 CUs
        const int target = 2048;
        split = ceil_div(target, blocks_i);
    }
    // each slice holds at least one tile of sources
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
    slice_len = ceil_div(slice_len, cfg.block) * cfg.block;
    cfg.n_split = ceil_div(n, slice_len);
    if (used) *used = cfg;

    const int ncomp = order == 2 ? 9 : 6;
    const int out0 = order == 3 ? 6 : 0;
    const int per_block = cfg.block * cfg.ipl;
    dim3 grid(ceil_div(n_act, per_block), cfg.n_split);
    const bool skipself = ctx->eps2 == 0.0;

    OutPtrs dst;
    int64_t slice_stride = 0;
    if (cfg.n_split == 1) {
        dst = out;
    } else {
        for (int c = 0; c < 12; ++c) dst.p[c] = nullptr;
        for (int c = 0; c < ncomp; ++c) dst.p[out0 + c] = ctx->partial + (int64_t)c * n_act;
        slice_stride = (int64_t)ncomp * n_act;
    }
    hipError_t e;
    if (order == 1)
        e = dispatch_shape<1>(cfg, skipself, grid, ctx->stream, src, active, n, n_act, ctx->eps2,
                              slice_len, dst, slice_stride);
    else if (order == 2)
        e = dispatch_shape<2>(cfg, skipself, grid, ctx->stream, src, active, n, n_act, ctx->eps2,
                              slice_len, dst, slice_stride);
    else
        e = dispatch_shape<3>(cfg, skipself, grid, ctx->stream, src, active, n, n_act, ctx->eps2,
                              slice_len, dst, slice_stride);
    if (e != hipSuccess || cfg.n_split == 1) return e;
    const int64_t total = (int64_t)ncomp * n_act;
    int rb = ceil_div(total, 256);
    if (rb > 4096) rb = 4096;
    hipLaunchKernelGGL(k_reduce_slices, dim3(rb), dim3(256), 0, ctx->stream, ctx->partial,
                       (int64_t)n_act, cfg.n_split, ncomp, out0, n_act, out);
    return hipGetLastError();
}

}  // namespace h6
