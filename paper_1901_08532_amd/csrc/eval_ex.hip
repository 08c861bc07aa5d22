// Extended-precision (EX) and single-precision (SP) evaluation of
// acceleration, jerk and snap (order 2).
//
// Sec. 3 item 6 of the paper lets the whole evaluation run in one of three
// arithmetics: IEEE double (DP), an extended type of about 48 significand
// bits with the single-precision exponent range (EX), or plain single
// precision (SP); its accuracy study compares the three by the drift of
// energy and angular momentum. These kernels are the EX and SP forms of the
// pair sum; the predictor, corrector and step rule stay FP64.
//
// EX is double-single ("float-float") arithmetic: a value is an unevaluated
// sum h + l of two floats with |l| <= ulp(h)/2, and every operation is built
// from error-free transformations of float operations:
//   TwoSum (Knuth): s = fl(a + b) and the exact error of that addition;
//   Fast2Sum (Dekker): the same when |a| >= |b|, in three operations;
//   TwoProd: p = fl(a b) and its exact error fma(a, b, -p).
// The differences of nearby coordinates use the accurate addition (TwoSum
// on both the high and the low parts, then two renormalisations), so that
// they keep their full double-single precision; the other sums (of
// products, and the accumulations) the sloppy one, whose operand-relative
// error is that of the terms it adds. Multiplication adds the two cross
// products into the error of the high product. The reciprocal square root
// starts from the hardware single-precision estimate and takes one
// third-order Newton step in double-single. Only float operations are used
// in the pair loop; FP64 inputs are split into (h, l) once when staged
// (h = fl32(x), l = fl32(x - h)) and the per-slice double-single sums leave
// the kernel as the exact double h + l. Contraction of a * b + c into one
// fused operation is switched off in the helpers: the error terms depend on
// each operation being rounded on its own.
//
// SP rounds the staged inputs to float and does every operation of the pair
// terms and the per-slice sums in float.
//
// Both use the FP64 kernel's launch structure: a tile of source records in
// LDS, one target per lane, the source sum split into slices across
// workgroups; the slices (at most a few dozen partial sums per target) are
// combined by the common compensated FP64 slice reduction.
#include "h6_internal.h"

namespace h6 {
namespace {

// ---------------------------------------------------------------- EX
struct fpair {
    float h, l;
};

__device__ __forceinline__ fpair two_sum(float a, float b) {
#pragma clang fp contract(off)
    const float s = a + b;
    const float bb = s - a;
    const float e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

__device__ __forceinline__ fpair fast_two_sum(float a, float b) {  // needs |a| >= |b| or a == 0
#pragma clang fp contract(off)
    const float s = a + b;
    const float e = b - (s - a);
    return {s, e};
}

__device__ __forceinline__ fpair two_prod(float a, float b) {
#pragma clang fp contract(off)
    const float p = a * b;
    return {p, fmaf(a, b, -p)};
}

__device__ __forceinline__ fpair ds_add(fpair x, fpair y) {
#pragma clang fp contract(off)
    fpair s = two_sum(x.h, y.h);
    const fpair t = two_sum(x.l, y.l);
    s.l += t.h;
    s = fast_two_sum(s.h, s.l);
    s.l += t.l;
    return fast_two_sum(s.h, s.l);
}

// The sum without the error-free addition of the low parts (the "sloppy"
// form, 11 operations against 20): exact sum of the high parts, the low
// parts and its error added in float, renormalised. Its error is about
// 2u^2 (|x| + |y|), u = 2^-24: relative to the result when x and y have
// the same sign, to the operands' size when they cancel. The pair terms
// carry operand-relative errors of that size anyway (every product, sum of
// products and accumulation is rounded relative to its operands), so it is
// used for those; the differences of nearby coordinates, whose relative
// precision the pair terms need, keep the accurate form.
__device__ __forceinline__ fpair ds_add_sloppy(fpair x, fpair y) {
#pragma clang fp contract(off)
    fpair s = two_sum(x.h, y.h);
    s.l += x.l + y.l;
    return fast_two_sum(s.h, s.l);
}

__device__ __forceinline__ fpair ds_neg(fpair x) { return {-x.h, -x.l}; }

__device__ __forceinline__ fpair ds_sub_sloppy(fpair x, fpair y) {
    return ds_add_sloppy(x, ds_neg(y));
}

__device__ __forceinline__ fpair ds_sub(fpair x, fpair y) { return ds_add(x, ds_neg(y)); }

__device__ __forceinline__ fpair ds_add_f(fpair x, float b) {
#pragma clang fp contract(off)
    fpair s = two_sum(x.h, b);
    s.l += x.l;
    return fast_two_sum(s.h, s.l);
}

__device__ __forceinline__ fpair ds_mul(fpair x, fpair y) {
#pragma clang fp contract(off)
    fpair p = two_prod(x.h, y.h);
    p.l = fmaf(x.h, y.l, fmaf(x.l, y.h, p.l));
    return fast_two_sum(p.h, p.l);
}

// Products that only feed a sloppy sum skip the final renormalisation: the
// sum adds the low parts in float and renormalises itself, so a low part a
// few ulp of the high one larger costs nothing measurable.
__device__ __forceinline__ fpair ds_mul_raw(fpair x, fpair y) {
#pragma clang fp contract(off)
    fpair p = two_prod(x.h, y.h);
    p.l = fmaf(x.h, y.l, fmaf(x.l, y.h, p.l));
    return p;
}

__device__ __forceinline__ fpair ds_sqr_raw(fpair x) {
#pragma clang fp contract(off)
    fpair p = two_prod(x.h, x.h);
    p.l = fmaf(x.h + x.h, x.l, p.l);
    return p;
}

__device__ __forceinline__ fpair ds_mul_f(fpair x, float b) {
#pragma clang fp contract(off)
    fpair p = two_prod(x.h, b);
    p.l = fmaf(x.l, b, p.l);
    return fast_two_sum(p.h, p.l);
}

__device__ __forceinline__ fpair ds_sqr(fpair x) {
#pragma clang fp contract(off)
    fpair p = two_prod(x.h, x.h);
    p.l = fmaf(x.h + x.h, x.l, p.l);
    return fast_two_sum(p.h, p.l);
}

// x times a power of two: exact
__device__ __forceinline__ fpair ds_scale2(fpair x, float p2) { return {x.h * p2, x.l * p2}; }

__device__ __forceinline__ fpair ds_from(double d) {
    const float h = (float)d;
    return {h, (float)(d - (double)h)};
}

__device__ __forceinline__ double ds_to_double(fpair x) { return (double)x.h + (double)x.l; }

// 1/sqrt(r2): single-precision estimate y0 (relative error d of a few
// 2^-24), then y = y0 (1 + e/2 + 3 e^2/8) with e = 1 - r2 y0^2 formed in
// double-single; the step leaves a relative error of about (5/2) d^3, below
// the double-single rounding. e^2 needs only float precision (it is of
// order d^2).
__device__ __forceinline__ fpair ds_rsqrt(fpair r2) {
#pragma clang fp contract(off)
    const float y0 = __builtin_amdgcn_rsqf(r2.h);
    const fpair y2 = two_prod(y0, y0);
    const fpair e = ds_add_f(ds_neg(ds_mul(r2, y2)), 1.0f);
    const float e2 = e.h * e.h * 0.375f;
    const fpair p = ds_add_f(ds_scale2(e, 0.5f), e2);
    return ds_add_f(ds_mul_f(p, y0), y0);
}

__device__ __forceinline__ fpair ds_dot3(const fpair *p, const fpair *q) {
    return ds_add_sloppy(ds_add_sloppy(ds_mul_raw(p[0], q[0]), ds_mul_raw(p[1], q[1])),
                         ds_mul_raw(p[2], q[2]));
}

// Pair terms of order 2 in double-single, added to acc[0..8]: with
// R^2 = |r|^2 + eps^2, alpha = r.v/R^2, beta = (v.v + r.a)/R^2 + alpha^2,
//   A = m r/R^3, J = m w/R^3 with w = v - 3 alpha r,
//   S = m u/R^3 with u = a - 6 alpha w - 3 beta r.
__device__ __forceinline__ void pair_ex(const fpair *r, const fpair *v, const fpair *a, fpair r2,
                                        fpair mj, fpair *acc) {
    const fpair rinv = ds_rsqrt(r2);
    const fpair rinv2 = ds_sqr(rinv);
    const fpair mr3 = ds_mul(ds_mul(mj, rinv), rinv2);
    const fpair alpha = ds_mul(ds_dot3(r, v), rinv2);
    const fpair a3 = ds_mul_f(alpha, 3.0f);
    fpair w[3], u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) w[c] = ds_sub_sloppy(v[c], ds_mul_raw(a3, r[c]));
    const fpair vvra = ds_add_sloppy(ds_dot3(v, v), ds_dot3(r, a));
    const fpair beta = ds_add_sloppy(ds_sqr_raw(alpha), ds_mul_raw(vvra, rinv2));
    const fpair b3 = ds_mul_f(beta, 3.0f);
    const fpair a6 = ds_scale2(a3, 2.0f);
#pragma unroll
    for (int c = 0; c < 3; ++c)
        u[c] = ds_sub_sloppy(ds_sub_sloppy(a[c], ds_mul_raw(a6, w[c])), ds_mul_raw(b3, r[c]));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[c] = ds_add_sloppy(acc[c], ds_mul_raw(mr3, r[c]));
        acc[3 + c] = ds_add_sloppy(acc[3 + c], ds_mul_raw(mr3, w[c]));
        acc[6 + c] = ds_add_sloppy(acc[6 + c], ds_mul_raw(mr3, u[c]));
    }
}

// Far, massless padding source: contributes exactly zero.
constexpr float kPadPosF = 1.0e18f;

// LDS record of one source: x, v, a and m as (h, l) pairs, five float4.
template <int BLOCK, bool SKIPSELF>
__global__ __launch_bounds__(BLOCK) void k_eval_ex(SrcPtrs src, const int32_t *__restrict__ active,
                                                   int n, int n_act, double eps2_d, int slice_len,
                                                   OutPtrs out, int64_t slice_stride) {
    __shared__ float4 tile[BLOCK * 5];
    const int tid = threadIdx.x;
    const int k = (int)blockIdx.x * BLOCK + tid;
    const int kc = k < n_act ? k : n_act - 1;
    const int p = active ? active[kc] : kc;
    fpair xi[3], vi[3], ai[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xi[c] = ds_from(src.x[c][p]);
        vi[c] = ds_from(src.v[c][p]);
        ai[c] = ds_from(src.a[c][p]);
    }
    const fpair eps2 = ds_from(eps2_d);
    fpair acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = {0.0f, 0.0f};

    const int jb = (int)blockIdx.y * slice_len;
    const int je = min(n, jb + slice_len);
    for (int jt = jb; jt < je; jt += BLOCK) {
        __syncthreads();
        {
            const int jj = jt + tid;
            float4 *rec = &tile[tid * 5];
            if (jj < je) {
                fpair f[10];
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    f[c] = ds_from(src.x[c][jj]);
                    f[3 + c] = ds_from(src.v[c][jj]);
                    f[6 + c] = ds_from(src.a[c][jj]);
                }
                f[9] = ds_from(src.m[jj]);
#pragma unroll
                for (int q = 0; q < 5; ++q)
                    rec[q] = make_float4(f[2 * q].h, f[2 * q].l, f[2 * q + 1].h, f[2 * q + 1].l);
            } else {
                rec[0] = make_float4(kPadPosF, 0.0f, kPadPosF, 0.0f);
                rec[1] = make_float4(kPadPosF, 0.0f, 0.0f, 0.0f);
#pragma unroll
                for (int q = 2; q < 5; ++q) rec[q] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        }
        __syncthreads();
        for (int q = 0; q < BLOCK; ++q) {
            const float4 *rec = &tile[q * 5];
            fpair f[10];
#pragma unroll
            for (int t = 0; t < 5; ++t) {
                const float4 d = rec[t];
                f[2 * t] = {d.x, d.y};
                f[2 * t + 1] = {d.z, d.w};
            }
            fpair r[3], v[3], a[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                r[c] = ds_sub(f[c], xi[c]);
                v[c] = ds_sub(f[3 + c], vi[c]);
                a[c] = ds_sub(f[6 + c], ai[c]);
            }
            fpair r2 = ds_add_sloppy(
                ds_add_sloppy(ds_add_sloppy(eps2, ds_sqr_raw(r[0])), ds_sqr_raw(r[1])),
                ds_sqr_raw(r[2]));
            fpair mj = f[9];
            if (SKIPSELF && (jt + q) == p) {  // r, v, a are zero: mask the 1/0
                r2 = {1.0f, 0.0f};
                mj = {0.0f, 0.0f};
            }
            pair_ex(r, v, a, r2, mj, acc);
        }
    }
    if (k < n_act) {
        const int64_t soff = (int64_t)blockIdx.y * slice_stride;
#pragma unroll
        for (int q = 0; q < 9; ++q) out.p[q][soff + k] = ds_to_double(acc[q]);
    }
}

// ---------------------------------------------------------------- SP
// LDS record of one source: x, v, a, m as floats (plus padding), three float4.
template <int BLOCK, bool SKIPSELF>
__global__ __launch_bounds__(BLOCK) void k_eval_sp(SrcPtrs src, const int32_t *__restrict__ active,
                                                   int n, int n_act, double eps2_d, int slice_len,
                                                   OutPtrs out, int64_t slice_stride) {
    __shared__ float4 tile[BLOCK * 3];
    const int tid = threadIdx.x;
    const int k = (int)blockIdx.x * BLOCK + tid;
    const int kc = k < n_act ? k : n_act - 1;
    const int p = active ? active[kc] : kc;
    float xi[3], vi[3], ai[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xi[c] = (float)src.x[c][p];
        vi[c] = (float)src.v[c][p];
        ai[c] = (float)src.a[c][p];
    }
    const float eps2 = (float)eps2_d;
    float acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0.0f;

    const int jb = (int)blockIdx.y * slice_len;
    const int je = min(n, jb + slice_len);
    for (int jt = jb; jt < je; jt += BLOCK) {
        __syncthreads();
        {
            const int jj = jt + tid;
            float4 *rec = &tile[tid * 3];
            if (jj < je) {
                rec[0] = make_float4((float)src.x[0][jj], (float)src.x[1][jj], (float)src.x[2][jj],
                                     (float)src.m[jj]);
                rec[1] = make_float4((float)src.v[0][jj], (float)src.v[1][jj], (float)src.v[2][jj],
                                     (float)src.a[0][jj]);
                rec[2] = make_float4((float)src.a[1][jj], (float)src.a[2][jj], 0.0f, 0.0f);
            } else {
                rec[0] = make_float4(kPadPosF, kPadPosF, kPadPosF, 0.0f);
                rec[1] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                rec[2] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
        }
        __syncthreads();
        for (int q = 0; q < BLOCK; ++q) {
            const float4 r0 = tile[q * 3], r1 = tile[q * 3 + 1], r2v = tile[q * 3 + 2];
            const float dx = r0.x - xi[0], dy = r0.y - xi[1], dz = r0.z - xi[2];
            const float dvx = r1.x - vi[0], dvy = r1.y - vi[1], dvz = r1.z - vi[2];
            const float dax = r1.w - ai[0], day = r2v.x - ai[1], daz = r2v.y - ai[2];
            float r2 = fmaf(dz, dz, fmaf(dy, dy, fmaf(dx, dx, eps2)));
            float mj = r0.w;
            if (SKIPSELF && (jt + q) == p) {
                r2 = 1.0f;
                mj = 0.0f;
            }
            // hardware estimate refined by one Newton step
            const float y0 = __builtin_amdgcn_rsqf(r2);
            const float rinv = y0 * fmaf(-0.5f * r2 * y0, y0, 1.5f);
            const float rinv2 = rinv * rinv;
            const float mr3 = mj * rinv * rinv2;
            const float alpha = fmaf(dz, dvz, fmaf(dy, dvy, dx * dvx)) * rinv2;
            const float a3 = 3.0f * alpha;
            const float wx = fmaf(-a3, dx, dvx), wy = fmaf(-a3, dy, dvy), wz = fmaf(-a3, dz, dvz);
            const float vvra =
                fmaf(dz, daz, fmaf(dy, day, fmaf(dx, dax, fmaf(dvz, dvz, fmaf(dvy, dvy, dvx * dvx)))));
            const float beta = fmaf(alpha, alpha, vvra * rinv2);
            const float b3 = 3.0f * beta, a6 = a3 + a3;
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
    }
    if (k < n_act) {
        const int64_t soff = (int64_t)blockIdx.y * slice_stride;
#pragma unroll
        for (int q = 0; q < 9; ++q) out.p[q][soff + k] = (double)acc[q];
    }
}

template <bool EX, bool SKIPSELF>
hipError_t launch_one(dim3 grid, hipStream_t st, const SrcPtrs &src, const int32_t *active, int n,
                      int n_act, double eps2, int slice_len, const OutPtrs &out,
                      int64_t slice_stride) {
    if constexpr (EX)
        hipLaunchKernelGGL((k_eval_ex<kExtBlock, SKIPSELF>), grid, dim3(kExtBlock), 0, st, src,
                           active, n, n_act, eps2, slice_len, out, slice_stride);
    else
        hipLaunchKernelGGL((k_eval_sp<kExtBlock, SKIPSELF>), grid, dim3(kExtBlock), 0, st, src,
                           active, n, n_act, eps2, slice_len, out, slice_stride);
    return hipGetLastError();
}

}  // namespace

hipError_t dispatch_ext(int precision, bool skipself, dim3 grid, hipStream_t st, const SrcPtrs &src,
                        const int32_t *active, int n, int n_act, double eps2, int slice_len,
                        const OutPtrs &out, int64_t slice_stride) {
    if (precision == H6_EX)
        return skipself ? launch_one<true, true>(grid, st, src, active, n, n_act, eps2, slice_len,
                                                 out, slice_stride)
                        : launch_one<true, false>(grid, st, src, active, n, n_act, eps2, slice_len,
                                                  out, slice_stride);
    if (precision == H6_SP)
        return skipself ? launch_one<false, true>(grid, st, src, active, n, n_act, eps2, slice_len,
                                                  out, slice_stride)
                        : launch_one<false, false>(grid, st, src, active, n, n_act, eps2,
                                                   slice_len, out, slice_stride);
    return hipErrorInvalidValue;
}

}  // namespace h6
