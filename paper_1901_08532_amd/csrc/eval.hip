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
#include <algorithm>
#include <climits>

#include "device_math.h"
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

// Pair terms of order 2 (a, j, s) accumulated into acc[0..8], from the
// differences source - target r, v, a and the source mass. With
// R^2 = |r|^2 + eps^2, alpha = r.v/R^2, beta = (v.v + r.a)/R^2 + alpha^2:
//   A = m r / R^3,  J = m w / R^3 with w = v - 3 alpha r,
//   S = m u / R^3 with u = a - 6 alpha w - 3 beta r.
__device__ __forceinline__ void pair_acc2(double dx, double dy, double dz, double dvx, double dvy,
                                          double dvz, double dax, double day, double daz,
                                          double r2, double mj, double *acc) {
    const double rinv = rsqrt_f64(r2);
    const double rinv2 = rinv * rinv;
    const double mr3 = (mj * rinv) * rinv2;
    const double rv = fma(dz, dvz, fma(dy, dvy, dx * dvx));
    const double alpha = rv * rinv2;
    const double a3 = 3.0 * alpha;
    const double wx = fma(-a3, dx, dvx), wy = fma(-a3, dy, dvy), wz = fma(-a3, dz, dvz);
    const double vvra =
        fma(dz, daz, fma(dy, day, fma(dx, dax, fma(dvz, dvz, fma(dvy, dvy, dvx * dvx)))));
    const double beta = fma(alpha, alpha, vvra * rinv2);
    const double b3 = 3.0 * beta;
    const double a6 = a3 + a3;
    const double ux = fma(-a6, wx, fma(-b3, dx, dax));
    const double uy = fma(-a6, wy, fma(-b3, dy, day));
    const double uz = fma(-a6, wz, fma(-b3, dz, daz));
    acc[0] = fma(mr3, dx, acc[0]);
    acc[1] = fma(mr3, dy, acc[1]);
    acc[2] = fma(mr3, dz, acc[2]);
    acc[3] = fma(mr3, wx, acc[3]);
    acc[4] = fma(mr3, wy, acc[4]);
    acc[5] = fma(mr3, wz, acc[5]);
    acc[6] = fma(mr3, ux, acc[6]);
    acc[7] = fma(mr3, uy, acc[7]);
    acc[8] = fma(mr3, uz, acc[8]);
}

// Far, massless padding source: contributes exactly zero.
constexpr double kPadPos = 1.0e18;

template <int ORDER, int BLOCK, int IPL, bool SKIPSELF>
__global__ __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(IPL == 1 ? 4 : 2))) void k_eval_f64(SrcPtrs src, const int32_t *__restrict__ active,
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
                if constexpr (ORDER == 2) {
                    pair_acc2(dx, dy, dz, dvx, dvy, dvz, aj0 - ai[u][0], aj1 - ai[u][1],
                              aj2 - ai[u][2], r2, m_eff, acc[u]);
                } else {
                    const double rinv = rsqrt_f64(r2);
                    const double rinv2 = rinv * rinv;
                    const double mr3 = (m_eff * rinv) * rinv2;
                    const double rv = fma(dz, dvz, fma(dy, dvy, dx * dvx));
                    const double alpha = rv * rinv2;
                    const double a3 = 3.0 * alpha;
                    // w = v - 3 alpha r, so that J = mr3 w
                    const double wx = fma(-a3, dx, dvx), wy = fma(-a3, dy, dvy),
                                 wz = fma(-a3, dz, dvz);
                    if constexpr (ORDER == 1) {
                        acc[u][0] = fma(mr3, dx, acc[u][0]);
                        acc[u][1] = fma(mr3, dy, acc[u][1]);
                        acc[u][2] = fma(mr3, dz, acc[u][2]);
                        acc[u][3] = fma(mr3, wx, acc[u][3]);
                        acc[u][4] = fma(mr3, wy, acc[u][4]);
                        acc[u][5] = fma(mr3, wz, acc[u][5]);
                    } else {
                        const double dax = aj0 - ai[u][0], day = aj1 - ai[u][1],
                                     daz = aj2 - ai[u][2];
                        const double djx = jj0 - ji[u][0], djy = jj1 - ji[u][1],
                                     djz = jj2 - ji[u][2];
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

// Evaluation for small active sets (order 2): the lanes of a wave run over
// sources (coalesced global loads, no LDS), each wave serving TPW targets
// whose predicted state is wave-uniform; per-lane sums are flushed into
// compensated pairs every kSmallFlush sources and combined across lanes by
// a fixed butterfly. Grid: (one wave per TPW targets) x (source slices).
constexpr int kSmallFlush = 16;

template <int TPW, bool SKIPSELF>
__global__ __launch_bounds__(64) void k_eval_small(SrcPtrs src, const int32_t *__restrict__ active,
                                                    int n, int n_act, double eps2, int slice_len,
                                                    OutPtrs out, int64_t slice_stride) {
    const int lane = threadIdx.x;
    const int wave = blockIdx.x;
    double xi[TPW][3], vi[TPW][3], ai[TPW][3];
    int pid[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        int k = wave * TPW + t;
        k = k < n_act ? k : n_act - 1;
        const int p = active ? active[k] : k;
        pid[t] = p;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xi[t][c] = src.x[c][p];
            vi[t][c] = src.v[c][p];
            ai[t][c] = src.a[c][p];
        }
    }
    double acc[TPW][9], hi[TPW][9], lo[TPW][9];
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int q = 0; q < 9; ++q) acc[t][q] = hi[t][q] = lo[t][q] = 0.0;

    const int jb = (int)blockIdx.y * slice_len;
    const int je = min(n, jb + slice_len);
    int since_flush = 0;
    for (int j = jb + lane; j < je; j += 64) {
        const double xj0 = src.x[0][j], xj1 = src.x[1][j], xj2 = src.x[2][j];
        const double vj0 = src.v[0][j], vj1 = src.v[1][j], vj2 = src.v[2][j];
        const double aj0 = src.a[0][j], aj1 = src.a[1][j], aj2 = src.a[2][j];
        const double mj = src.m[j];
#pragma unroll
        for (int t = 0; t < TPW; ++t) {
            const double dx = xj0 - xi[t][0], dy = xj1 - xi[t][1], dz = xj2 - xi[t][2];
            double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
            double m_eff = mj;
            if (SKIPSELF) {
                const bool self = j == pid[t];
                r2 = self ? 1.0 : r2;
                m_eff = self ? 0.0 : mj;
            }
            pair_acc2(dx, dy, dz, vj0 - vi[t][0], vj1 - vi[t][1], vj2 - vi[t][2], aj0 - ai[t][0],
                      aj1 - ai[t][1], aj2 - ai[t][2], r2, m_eff, acc[t]);
        }
        if (++since_flush == kSmallFlush) {
            since_flush = 0;
#pragma unroll
            for (int t = 0; t < TPW; ++t)
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    two_sum_into(hi[t][q], lo[t][q], acc[t][q]);
                    acc[t][q] = 0.0;
                }
        }
    }
    const int64_t soff = (int64_t)blockIdx.y * slice_stride;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            two_sum_into(hi[t][q], lo[t][q], acc[t][q]);
            double sv = hi[t][q], cv = lo[t][q];
            wave_comp_sum(sv, cv);
            const int k = wave * TPW + t;
            if (lane == 0 && k < n_act) out.p[q][soff + k] = sv + cv;
        }
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
    (void)precision;
    EvalConfig cfg;
    const int small_max = ctx->cfg_small >= 0 ? ctx->cfg_small : kDefaultSmallMax;
    if (order == 2 && n_act <= small_max) {
        // source-parallel kernel: one wave per TPW targets
        cfg.kind = 1;
        cfg.block = 64;
        cfg.ipl = n_act <= 4 ? 1 : 2;
        const int waves_i = ceil_div(n_act, cfg.ipl);
        int split = ceil_div(kTargetWaves, waves_i);
        const int max_split = ceil_div(n, kSmallMinSlice);
        if (split > max_split) split = max_split;
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
        cfg.ipl = ctx->cfg_ipl ? ctx->cfg_ipl : (n_act <= 512 ? 1 : 2);
    }
    const int per_block = cfg.block * cfg.ipl;
    const int blocks_i = ceil_div(n_act, per_block);
    int split;
    if (ctx->cfg_split && order == 2) {
        split = ctx->cfg_split;
    } else {
        // measured footprints on gfx950: order 2 with one target per lane
        // <= 128 VGPRs (4 waves per SIMD), two per lane <= 256 (2 waves);
        // start-up passes <= 128
        const int waves_per_simd = (order == 2 && cfg.ipl == 2) ? 2 : 4;
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
    const bool skipself = ctx->eps2 == 0.0;

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
    if (order == 2 && precision == H6_MIXED) {
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
