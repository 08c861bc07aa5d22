// Bodies of the mixed-precision a/j/s evaluation kernels, shared by the
// host-shaped launches (eval_mixed.hip) and the device-resident block loop
// (blockloop.hip). See eval_mixed.hip for the design.
#pragma once

#include "device_math.h"
#include "eval_body.h"
#include "h6_internal.h"

namespace h6 {
namespace mixedbody {

// Far, massless padding source: contributes exactly zero; small enough that
// its squared distance stays finite in FP32.
constexpr double kPadPosMixed = 1.0e15;
// Sources per FP32 partial sum before it joins the FP64 sums. Longer
// partial sums are cheaper (64 sources: a mixed block-step interval at
// N = 262144 about 5% faster, the largest a/j/s errors against the oracle
// unchanged) but their round-off dominates the energy error of fixed-step
// runs: N = 4096, 8 time units, largest |dE/E| 1.8e-11 with 8 sources,
// 3.5e-11 to 6.5e-11 with 16 to 64.
constexpr int kChunk = 8;

// Pair terms of order 2 in FP32, accumulated into acc[0..8] (FP32). Same
// factorisation as the FP64 routine: A = m r/R^3, J = m w/R^3 with
// w = v - 3 alpha r, S = m u/R^3 with u = a - 6 alpha w - 3 beta r.
__device__ __forceinline__ void pair_acc2_f32(float dx, float dy, float dz, float dvx, float dvy,
                                              float dvz, float dax, float day, float daz, float r2,
                                              float mj, float *acc) {
    // hardware estimate plus one Newton step: the estimate's own error is
    // not centred on zero, and a common bias of every pair term would show
    // as a secular energy drift
    const float y = __builtin_amdgcn_rsqf(r2);
    const float e = fmaf(-(r2 * y), y, 1.0f);
    const float rinv = fmaf(0.5f * y, e, y);
    const float rinv2 = rinv * rinv;
    const float mr3 = (mj * rinv) * rinv2;
    const float rv = fmaf(dz, dvz, fmaf(dy, dvy, dx * dvx));
    const float alpha = rv * rinv2;
    const float a3 = 3.0f * alpha;
    const float wx = fmaf(-a3, dx, dvx), wy = fmaf(-a3, dy, dvy), wz = fmaf(-a3, dz, dvz);
    const float vvra =
        fmaf(dz, daz, fmaf(dy, day, fmaf(dx, dax, fmaf(dvz, dvz, fmaf(dvy, dvy, dvx * dvx)))));
    const float beta = fmaf(alpha, alpha, vvra * rinv2);
    const float b3 = 3.0f * beta;
    const float a6 = a3 + a3;
    const float ux = fmaf(-a6, wx, fmaf(-b3, dx, dax));
    const float uy = fmaf(-a6, wy, fmaf(-b3, dy, day));
    const float uz = fmaf(-a6, wz, fmaf(-b3, dz, daz));
    acc[0] = fmaf(mr3, dx, acc[0]);
    acc[1] = fmaf(mr3, dy, acc[1]);
    acc[2] = fmaf(mr3, dz, acc[2]);
    acc[3] = fmaf(mr3, wx, acc[3]);
    acc[4] = fmaf(mr3, wy, acc[4]);
    acc[5] = fmaf(mr3, wz, acc[5]);
    acc[6] = fmaf(mr3, ux, acc[6]);
    acc[7] = fmaf(mr3, uy, acc[7]);
    acc[8] = fmaf(mr3, uz, acc[8]);
}

// LDS source record: x0 x1 | x2 v0 | v1 v2 (FP64), then a0 a1 a2 m (FP32).
struct alignas(16) RecMixed {
    double2 p0, p1, p2;
    float4 am;
};

// Body for the workgroup owning target block ib and source slice sl.
// tile: BLOCK records of workgroup memory.
template <int BLOCK, int IPL, bool SKIPSELF, class SRC>
__device__ __forceinline__ void mixed_tile_body(const SRC &S, int n, int n_act, double eps2,
                                                int slice_len, const OutPtrs &out,
                                                int64_t slice_stride, int ib, int sl,
                                                RecMixed *tile) {
    const int tid = threadIdx.x;
    const float eps2f = (float)eps2;

    double xi[IPL][3], vi[IPL][3];
    float ai[IPL][3];
    int pid[IPL], kid[IPL];
#pragma unroll
    for (int u = 0; u < IPL; ++u) {
        const int k = (ib * IPL + u) * BLOCK + tid;
        kid[u] = k;
        const int kc = k < n_act ? k : n_act - 1;
        const int p = S.target(kc);
        pid[u] = p;
        double ad[3], jd[3];
        S.template get<2>(p, xi[u], vi[u], ad, jd);
#pragma unroll
        for (int c = 0; c < 3; ++c) ai[u][c] = (float)ad[c];
    }
    // FP64 sums of the FP32 chunk sums, uncompensated: their rounding (about
    // 1e-16 relative per addition) stays orders of magnitude below the
    // FP32 pair terms' own (about 6e-8)
    double acc[IPL][9];
#pragma unroll
    for (int u = 0; u < IPL; ++u)
#pragma unroll
        for (int q = 0; q < 9; ++q) acc[u][q] = 0.0;

    const int jb = sl * slice_len;
    const int je = min(n, jb + slice_len);
    for (int jt = jb; jt < je; jt += BLOCK) {
        __syncthreads();
        {
            const int jj = jt + tid;
            RecMixed r;
            if (jj < je) {
                double xs[3], vs[3], as[3], jd[3];
                S.template get<2>(jj, xs, vs, as, jd);
                r.p0 = make_double2(xs[0], xs[1]);
                r.p1 = make_double2(xs[2], vs[0]);
                r.p2 = make_double2(vs[1], vs[2]);
                r.am = make_float4((float)as[0], (float)as[1], (float)as[2], (float)S.mass(jj));
            } else {
                r.p0 = make_double2(kPadPosMixed, kPadPosMixed);
                r.p1 = make_double2(kPadPosMixed, 0.0);
                r.p2 = make_double2(0.0, 0.0);
                r.am = make_float4(0.f, 0.f, 0.f, 0.f);
            }
            tile[tid] = r;
        }
        __syncthreads();

        for (int q0 = 0; q0 < BLOCK; q0 += kChunk) {
            float acc32[IPL][9];
#pragma unroll
            for (int u = 0; u < IPL; ++u)
#pragma unroll
                for (int q = 0; q < 9; ++q) acc32[u][q] = 0.0f;
#pragma unroll
            for (int qq = 0; qq < kChunk; ++qq) {
                const RecMixed r = tile[q0 + qq];
#pragma unroll
                for (int u = 0; u < IPL; ++u) {
                    const float dx = (float)(r.p0.x - xi[u][0]);
                    const float dy = (float)(r.p0.y - xi[u][1]);
                    const float dz = (float)(r.p1.x - xi[u][2]);
                    const float dvx = (float)(r.p1.y - vi[u][0]);
                    const float dvy = (float)(r.p2.x - vi[u][1]);
                    const float dvz = (float)(r.p2.y - vi[u][2]);
                    float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2f)));
                    float m_eff = r.am.w;
                    if (SKIPSELF) {
                        const bool self = (jt + q0 + qq) == pid[u];
                        r2 = self ? 1.0f : r2;
                        m_eff = self ? 0.0f : m_eff;
                    }
                    pair_acc2_f32(dx, dy, dz, dvx, dvy, dvz, r.am.x - ai[u][0], r.am.y - ai[u][1],
                                  r.am.z - ai[u][2], r2, m_eff, acc32[u]);
                }
            }
#pragma unroll
            for (int u = 0; u < IPL; ++u)
#pragma unroll
                for (int q = 0; q < 9; ++q) acc[u][q] += (double)acc32[u][q];
        }
    }
    const int64_t soff = (int64_t)sl * slice_stride;
#pragma unroll
    for (int u = 0; u < IPL; ++u)
        if (kid[u] < n_act)
#pragma unroll
            for (int q = 0; q < 9; ++q) out.p[q][soff + kid[u] * out.kstride] = acc[u][q];
}

// Small active sets: lanes over sources, TPW targets per wave (as the FP64
// source-parallel kernel, passes of PASS sources per lane with their loads
// issued together; fewer for a kernel that must fit four waves per SIMD),
// FP32 pair arithmetic, FP32 partial sums over kChunk sources per lane
// added to FP64 sums.
constexpr int kPassM = 4;

// red: 64 * 9 * TPW doubles of workgroup memory (the final reduction).
template <int TPW, bool SKIPSELF, int PASS = kPassM, class SRC>
__device__ __forceinline__ void mixed_small_body(const SRC &S, int n, int n_act, double eps2,
                                                 int slice_len, const OutPtrs &out,
                                                 int64_t slice_stride, int wave, int sl,
                                                 double *red) {
    static_assert(kChunk % PASS == 0, "flush on pass boundaries");
    const int lane = threadIdx.x & 63;
    const float eps2f = (float)eps2;
    const int jb = sl * slice_len;
    const int je = min(n, jb + slice_len);
    // sources of one pass: independent of the targets, so the first pass is
    // fetched before the targets' (list, then state) loads
    auto load_pass = [&](int jp, double (*xs)[3], double (*vs)[3], float (*as)[3], float *ms) {
#pragma unroll
        for (int u = 0; u < PASS; ++u) {
            const int j = jp + u * 64 + lane;
            if (j < je) {
                double ad[3], jd[3];
                S.template get<2>(j, xs[u], vs[u], ad, jd);
#pragma unroll
                for (int c = 0; c < 3; ++c) as[u][c] = (float)ad[c];
                ms[u] = (float)S.mass(j);
            } else {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    xs[u][c] = kPadPosMixed;
                    vs[u][c] = 0.0;
                    as[u][c] = 0.0f;
                }
                ms[u] = 0.0f;
            }
        }
    };
    double xs[PASS][3], vs[PASS][3];
    float as[PASS][3], ms[PASS];
    load_pass(jb, xs, vs, as, ms);
    double xi[TPW][3], vi[TPW][3];
    float ai[TPW][3];
    int pid[TPW];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        int k = wave * TPW + t;
        k = k < n_act ? k : n_act - 1;
        const int p = S.target(k);
        pid[t] = p;
        double ad[3], jd[3];
        S.template get<2>(p, xi[t], vi[t], ad, jd);
#pragma unroll
        for (int c = 0; c < 3; ++c) ai[t][c] = (float)ad[c];
    }
    // FP32 sums over kChunk sources per lane, added to plain FP64 sums (as
    // in the tiled body)
    float acc32[TPW][9];
    double acc[TPW][9];
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            acc32[t][q] = 0.0f;
            acc[t][q] = 0.0;
        }
    int since_flush = 0;
    for (int jp = jb; jp < je; jp += PASS * 64) {
        if (jp != jb) load_pass(jp, xs, vs, as, ms);
#pragma unroll
        for (int u = 0; u < PASS; ++u) {
            const int j = jp + u * 64 + lane;
#pragma unroll
            for (int t = 0; t < TPW; ++t) {
                const float dx = (float)(xs[u][0] - xi[t][0]), dy = (float)(xs[u][1] - xi[t][1]),
                            dz = (float)(xs[u][2] - xi[t][2]);
                float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2f)));
                float m_eff = ms[u];
                if (SKIPSELF) {
                    const bool self = j == pid[t];
                    r2 = self ? 1.0f : r2;
                    m_eff = self ? 0.0f : m_eff;
                }
                pair_acc2_f32(dx, dy, dz, (float)(vs[u][0] - vi[t][0]),
                              (float)(vs[u][1] - vi[t][1]), (float)(vs[u][2] - vi[t][2]),
                              as[u][0] - ai[t][0], as[u][1] - ai[t][1], as[u][2] - ai[t][2], r2,
                              m_eff, acc32[t]);
            }
        }
        since_flush += PASS;
        if (since_flush == kChunk) {
            since_flush = 0;
#pragma unroll
            for (int t = 0; t < TPW; ++t)
#pragma unroll
                for (int q = 0; q < 9; ++q) {
                    acc[t][q] += (double)acc32[t][q];
                    acc32[t][q] = 0.0f;
                }
        }
    }
#pragma unroll
    for (int t = 0; t < TPW; ++t)
#pragma unroll
        for (int q = 0; q < 9; ++q) red[(t * 9 + q) * 64 + lane] = acc[t][q] + (double)acc32[t][q];
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
template <int BLOCK, int IPL, bool SKIPSELF>
__device__ __forceinline__ void mixed_tile_body(const SrcPtrs &src,
                                                const int32_t *__restrict__ active, int n,
                                                int n_act, double eps2, int slice_len,
                                                const OutPtrs &out, int64_t slice_stride, int ib,
                                                int sl) {
    __shared__ RecMixed tile[BLOCK];
    mixed_tile_body<BLOCK, IPL, SKIPSELF>(evalbody::PredSrc{src, active}, n, n_act, eps2,
                                          slice_len, out, slice_stride, ib, sl, tile);
}

template <int TPW, bool SKIPSELF>
__device__ __forceinline__ void mixed_small_body(const SrcPtrs &src,
                                                 const int32_t *__restrict__ active, int n,
                                                 int n_act, double eps2, int slice_len,
                                                 const OutPtrs &out, int64_t slice_stride,
                                                 int wave, int sl) {
    __shared__ double red[64 * 9 * TPW];
    mixed_small_body<TPW, SKIPSELF>(evalbody::PredSrc{src, active}, n, n_act, eps2, slice_len,
                                    out, slice_stride, wave, sl, red);
}

}  // namespace mixedbody
}  // namespace h6
