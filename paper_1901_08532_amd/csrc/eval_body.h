// Bodies of the a/j/s evaluation kernels (FP64), shared by the launches
// whose shape the host chooses (eval.hip) and the device-resident block
// loop (blockloop.hip). See eval.hip for the design.
#pragma once

#include "device_math.h"
#include "h6_internal.h"

namespace h6 {
namespace evalbody {

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

// Where a body finds its targets and sources. Every body takes a policy
// object with
//   int target(int k)             particle index of target rank k
//   void get<ORDER>(p, x, v, a, j) the (predicted) x, v, and for ORDER >= 2
//                                 a, for ORDER 3 j, of particle p
//   double mass(int p)
// PredSrc reads predicted arrays and an optional active list (NULL: rank k
// is particle k).
struct PredSrc {
    SrcPtrs src;
    const int32_t *active;
    __device__ __forceinline__ int target(int k) const { return active ? active[k] : k; }
    template <int ORDER>
    __device__ __forceinline__ void get(int p, double *x, double *v, double *a, double *j) const {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[c] = src.x[c][p];
            v[c] = src.v[c][p];
            a[c] = ORDER >= 2 ? src.a[c][p] : 0.0;
            j[c] = ORDER >= 3 ? src.j[c][p] : 0.0;
        }
    }
    __device__ __forceinline__ double mass(int p) const { return src.m[p]; }
};

// Body of the target-parallel LDS-tiled evaluation for the workgroup that
// owns target block ib (BLOCK * IPL targets) and source slice sl.
// tile: BLOCK * Traits<ORDER>::NREC double2 of workgroup memory. AHEAD
// (order 2, one target per lane, kernels with registers to spare): the next
// tile's source record is loaded while this tile's sums run, so that its
// latency is hidden.
template <int ORDER, int BLOCK, int IPL, bool SKIPSELF, bool AHEAD, class SRC>
__device__ __forceinline__ void eval_tile_body(const SRC &S, int n, int n_act, double eps2,
                                               int slice_len, const OutPtrs &out,
                                               int64_t slice_stride, int ib, int sl,
                                               double2 *tile) {
    using T = Traits<ORDER>;
    constexpr int NREC = T::NREC;
    constexpr int NACC = T::NACC;
    const int tid = threadIdx.x;

    // ---- targets: predicted state of particle active[k]
    double xi[IPL][3], vi[IPL][3], ai[IPL][3], ji[IPL][3];
    int pid[IPL], kid[IPL];
#pragma unroll
    for (int u = 0; u < IPL; ++u) {
        int k = (ib * IPL + u) * BLOCK + tid;
        kid[u] = k;
        int kc = k < n_act ? k : n_act - 1;
        int p = S.target(kc);
        pid[u] = p;
        S.template get<ORDER>(p, xi[u], vi[u], ai[u], ji[u]);
    }

    double acc[IPL][NACC], hi[IPL][NACC], lo[IPL][NACC];
#pragma unroll
    for (int u = 0; u < IPL; ++u)
#pragma unroll
        for (int q = 0; q < NACC; ++q) acc[u][q] = hi[u][q] = lo[u][q] = 0.0;

    const int jb = sl * slice_len;
    const int je = min(n, jb + slice_len);

    // this thread's source record of the tile starting at jt (far massless
    // padding past the slice end)
    auto fetch = [&](int jt, double2 *rec) {
        const int jj = jt + tid;
        if (jj < je) {
            double xs[3], vs[3], as[3], js[3];
            S.template get<ORDER>(jj, xs, vs, as, js);
            rec[0] = make_double2(xs[0], xs[1]);
            rec[1] = make_double2(xs[2], S.mass(jj));
            rec[2] = make_double2(vs[0], vs[1]);
            if (ORDER == 1) {
                rec[3] = make_double2(vs[2], 0.0);
            } else {
                rec[3] = make_double2(vs[2], as[0]);
                rec[4] = make_double2(as[1], as[2]);
            }
            if (ORDER == 3) {
                rec[5] = make_double2(js[0], js[1]);
                rec[6] = make_double2(js[2], 0.0);
            }
        } else {
            rec[0] = make_double2(kPadPos, kPadPos);
            rec[1] = make_double2(kPadPos, 0.0);
#pragma unroll
            for (int q = 2; q < NREC; ++q) rec[q] = make_double2(0.0, 0.0);
        }
    };
    constexpr bool kAhead = AHEAD && IPL == 1 && ORDER == 2;
    double2 ahead[NREC];
    if (kAhead && jb < je) fetch(jb, ahead);

    for (int jt = jb; jt < je; jt += BLOCK) {
        __syncthreads();  // previous tile fully consumed
        {
            double2 *rec = &tile[tid * NREC];
            if constexpr (kAhead) {
#pragma unroll
                for (int q = 0; q < NREC; ++q) rec[q] = ahead[q];
                if (jt + BLOCK < je) fetch(jt + BLOCK, ahead);
            } else {
                double2 cur[NREC];
                fetch(jt, cur);
#pragma unroll
                for (int q = 0; q < NREC; ++q) rec[q] = cur[q];
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

    const int64_t soff = (int64_t)sl * slice_stride;
#pragma unroll
    for (int u = 0; u < IPL; ++u) {
        if (kid[u] < n_act) {
#pragma unroll
            for (int q = 0; q < NACC; ++q)
                out.p[T::OUT0 + q][soff + kid[u] * out.kstride] = hi[u][q] + lo[u][q];
        }
    }
}

// Evaluation for small active sets (order 2): the lanes of a wave run over
// sources (coalesced global loads, no LDS), each wave serving TPW targets
// whose predicted state is wave-uniform. Each pass takes kSmallPass sources
// per lane, their loads issued together (sources past the slice end are the
// far massless padding); per-lane sums are flushed into compensated pairs
// every kSmallFlush passes and combined across lanes by a fixed butterfly,
// all 9 * TPW sums stage by stage. Grid: (one wave per TPW targets) x
// (source slices).
constexpr int kSmallPass = 4;
constexpr int kSmallFlush = 4;

// red: 64 * 9 * TPW doubles of workgroup memory (the final reduction).
template <int TPW, bool SKIPSELF, class SRC>
__device__ __forceinline__ void eval_small_body(const SRC &S, int n, int n_act, double eps2,
                                                int slice_len, const OutPtrs &out,
                                                int64_t slice_stride, int wave, int sl,
                                                double *red) {
    constexpr int PASS = TPW == 1 ? kSmallPass : kSmallPass / 2;  // register budget
    const int lane = threadIdx.x & 63;
    const int jb = sl * slice_len;
    const int je = min(n, jb + slice_len);
    // sources of one pass: their loads do not depend on the targets, so the
    // first pass is fetched before the targets' (list, then state) loads
    auto load_pass = [&](int jp, double (*xs)[3], double (*vs)[3], double (*as)[3], double *ms) {
#pragma unroll
        for (int u = 0; u < PASS; ++u) {
            const int j = jp + u * 64 + lane;
            if (j < je) {
                double jd[3];
                S.template get<2>(j, xs[u], vs[u], as[u], jd);
                ms[u] = S.mass(j);
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xs[u][c] = kPadPos;
                    vs[u][c] = as[u][c] = 0.0;
                }
                ms[u] = 0.0;
            }
        }
    };
    double xs[PASS][3], vs[PASS][3], as[PASS][3], ms[PASS];
    load_pass(jb, xs, vs, as, ms);
    double xi[TPW][3], vi[TPW][3], ai[TPW][3];
    int pid[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        int k = wave * TPW + t;
        k = k < n_act ? k : n_act - 1;
        const int p = S.target(k);
        pid[t] = p;
        double jd[3];
        S.template get<2>(p, xi[t], vi[t], ai[t], jd);
    }
    double acc[TPW][9], hi[TPW][9], lo[TPW][9];
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int q = 0; q < 9; ++q) acc[t][q] = hi[t][q] = lo[t][q] = 0.0;

    int passes = 0;
    for (int jp = jb; jp < je; jp += PASS * 64) {
        if (jp != jb) load_pass(jp, xs, vs, as, ms);
#pragma unroll
        for (int u = 0; u < PASS; ++u) {
            const int j = jp + u * 64 + lane;
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const double dx = xs[u][0] - xi[t][0], dy = xs[u][1] - xi[t][1],
                             dz = xs[u][2] - xi[t][2];
                double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
                double m_eff = ms[u];
                if (SKIPSELF) {
                    const bool self = j == pid[t];
                    r2 = self ? 1.0 : r2;
                    m_eff = self ? 0.0 : m_eff;
                }
                pair_acc2(dx, dy, dz, vs[u][0] - vi[t][0], vs[u][1] - vi[t][1],
                          vs[u][2] - vi[t][2], as[u][0] - ai[t][0], as[u][1] - ai[t][1],
                          as[u][2] - ai[t][2], r2, m_eff, acc[t]);
            }
        }
        if (++passes == kSmallFlush) {
            passes = 0;
#pragma unroll
            for (int t = 0; t < TPW; ++t)
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    two_sum_into(hi[t][q], lo[t][q], acc[t][q]);
                    acc[t][q] = 0.0;
                }
        }
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            two_sum_into(hi[t][q], lo[t][q], acc[t][q]);
            red[(t * 9 + q) * 64 + lane] = hi[t][q] + lo[t][q];
        }
    // totals over the lanes: lane t * 9 + q holds component q of target t
    const double total = wave_totals_lds<TPW * 9>(red);
    const int64_t soff = (int64_t)sl * slice_stride;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const int k = wave * TPW + t;
#pragma unroll
        for (int q = 0; q < 9; ++q)
            if (lane == t * 9 + q && k < n_act) out.p[q][soff + k * out.kstride] = total;
    }
}

// The bodies over predicted arrays (the host-shaped launches).
template <int ORDER, int BLOCK, int IPL, bool SKIPSELF>
__device__ __forceinline__ void eval_tile_body(const SrcPtrs &src,
                                               const int32_t *__restrict__ active, int n,
                                               int n_act, double eps2, int slice_len,
                                               const OutPtrs &out, int64_t slice_stride, int ib,
                                               int sl) {
    __shared__ double2 tile[BLOCK * Traits<ORDER>::NREC];
    eval_tile_body<ORDER, BLOCK, IPL, SKIPSELF, false>(PredSrc{src, active}, n, n_act, eps2,
                                                       slice_len, out, slice_stride, ib, sl, tile);
}

template <int TPW, bool SKIPSELF>
__device__ __forceinline__ void eval_small_body(const SrcPtrs &src,
                                                const int32_t *__restrict__ active, int n,
                                                int n_act, double eps2, int slice_len,
                                                const OutPtrs &out, int64_t slice_stride,
                                                int wave, int sl) {
    __shared__ double red[64 * 9 * TPW];
    eval_small_body<TPW, SKIPSELF>(PredSrc{src, active}, n, n_act, eps2, slice_len, out,
                                   slice_stride, wave, sl, red);
}

}  // namespace evalbody
}  // namespace h6
