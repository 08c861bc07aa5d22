// Per-particle bodies of the predictor and corrector, shared by the
// host-sequenced steps (steps.hip) and the device-resident block loop
// (blockloop.hip).
#pragma once

#include "device_math.h"
#include "h6_internal.h"

namespace h6 {
namespace stepbody {

constexpr double kTick = 1.0 / (double)((int64_t)1 << kTickBits);  // 2^-40

__device__ __forceinline__ int ceil_div_dev(int a, int b) { return (a + b - 1) / b; }

// Smallest level L >= lev_min with 2^(-k L) <= q, for q = (dt_crit)^k:
// with q = f 2^e, f in [0.5, 1), the condition is -k L <= e - 1, so
// L = ceil((1 - e) / k). q == 0 gives lev_cap (no admissible step);
// q NaN or +inf gives lev_min.
__device__ __forceinline__ int level_from_power(double q, int k, int lev_min, int lev_cap) {
    if (!(q == q) || q == __builtin_inf()) return lev_min;
    if (q <= 0.0) return lev_cap;
    int e;
    frexp(q, &e);
    const int p = 1 - e;  // L = ceil(p / k)
    int L = p >= 0 ? (p + k - 1) / k : -((-p) / k);
    if (L < lev_min) L = lev_min;
    if (L > lev_cap) L = lev_cap;
    return L;
}

__device__ __forceinline__ int level_of_ticks(int64_t dt) {
    return kTickBits - (63 - __builtin_clzll((unsigned long long)dt));
}

__device__ __forceinline__ double norm3(double a, double b, double c) {
    return sqrt(fma(a, a, fma(b, b, c * c)));
}

// ---------------------------------------------------------------- predictor
// Taylor prediction of one component over interval d: x to 5th order, v to
// 4th, a to 3rd, Horner form.
__device__ __forceinline__ void predict_comp(double x, double v, double a, double j, double s,
                                             double cr, double d, double &xo, double &vo,
                                             double &ao) {
    // a_p = a + d (j + d/2 (s + d/3 c))
    ao = fma(d, fma(d * 0.5, fma(d * (1.0 / 3.0), cr, s), j), a);
    // v_p = v + d (a + d/2 (j + d/3 (s + d/4 c)))
    vo = fma(d, fma(d * 0.5, fma(d * (1.0 / 3.0), fma(d * 0.25, cr, s), j), a), v);
    // x_p = x + d (v + d/2 (a + d/3 (j + d/4 (s + d/5 c))))
    xo = fma(d, fma(d * 0.5, fma(d * (1.0 / 3.0), fma(d * 0.25, fma(d * 0.2, cr, s), j), a), v),
             x);
}

// Taylor prediction of particle i over interval d.
__device__ __forceinline__ void predict_vals(const h6_state &st, int i, double d, double *xo,
                                             double *vo, double *ao) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
        predict_comp(st.x[c][i], st.v[c][i], st.a[c][i], st.j[c][i], st.s[c][i], st.c[c][i], d,
                     xo[c], vo[c], ao[c]);
}

__device__ __forceinline__ void predict_one(const h6_state &st, int i, double d,
                                            const h6_pred &out) {
    double xp[3], vp[3], ap[3];
    predict_vals(st, i, d, xp, vp, ap);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        out.x[c][i] = xp[c];
        out.v[c][i] = vp[c];
        out.a[c][i] = ap[c];
    }
}

// ---------------------------------------------------------------- corrector
// State of one particle before its correction.
struct OldState {
    double x[3], v[3], a[3], j[3], s[3];
    int64_t dt;
};

template <bool SHARED>
__device__ __forceinline__ OldState load_old(const h6_state &st, int i) {
    OldState o;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        o.x[c] = st.x[c][i];
        o.v[c] = st.v[c][i];
        o.a[c] = st.a[c][i];
        o.j[c] = st.j[c][i];
        o.s[c] = st.s[c][i];
    }
    o.dt = SHARED ? 0 : st.dt[i];
    return o;
}

// 6th-order Hermite corrector, quintic interpolation of crackle, pop and
// the fifth derivative at the step end, and the power-of-two step rule.
// Computes, for a particle with old state o and the new a1, j1, s1 (fa, fj,
// fs), the corrected x1, v1 and the interpolated crackle c1; block steps
// (SHARED false) also the new level (step 2^-level), taking the step from
// o.dt.
template <bool SHARED>
__device__ __forceinline__ void correct_from(const OldState &o, const double *fa,
                                             const double *fj, const double *fs, int64_t t_next,
                                             double dt_sh, double eta6, int lev_min, int lev_max,
                                             int32_t *flags, double *x1o, double *v1o,
                                             double *c1o, int *lev_out) {
    const int64_t dt_old = o.dt;
    const double h = SHARED ? dt_sh : (double)dt_old * kTick;
    const double h2 = h * h;
    const double hinv = 1.0 / h;
    const double hinv2 = hinv * hinv, hinv3 = hinv2 * hinv;
    double pn[3], dn[3];
    bool finite = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double x0 = o.x[c], v0 = o.v[c];
        const double a0 = o.a[c], j0 = o.j[c], s0 = o.s[c];
        const double a1 = fa[c], j1 = fj[c], s1 = fs[c];
        // v1 = v0 + h/2 (a0 + a1) - h^2/10 (j1 - j0) + h^3/120 (s0 + s1)
        const double v1 =
            v0 + h * fma(h, fma(h * (1.0 / 120.0), s0 + s1, -0.1 * (j1 - j0)), 0.5 * (a0 + a1));
        // x1 = x0 + h/2 (v0 + v1) - h^2/10 (a1 - a0) + h^3/120 (j0 + j1)
        const double x1 =
            x0 + h * fma(h, fma(h * (1.0 / 120.0), j0 + j1, -0.1 * (a1 - a0)), 0.5 * (v0 + v1));
        const double da = a1 - a0;
        // derivatives of the quintic through (a, j, s) at both ends, at the end
        const double c1 = fma(h2, 9.0 * s1 - 3.0 * s0, fma(-h, fma(24.0, j0, 36.0 * j1), 60.0 * da)) * hinv3;
        x1o[c] = x1;
        v1o[c] = v1;
        c1o[c] = c1;
        finite = finite && isfinite(x1) && isfinite(v1) && isfinite(c1);
        if (!SHARED) {
            pn[c] = fma(h2, 36.0 * s1 - 24.0 * s0, fma(-h, fma(168.0, j0, 192.0 * j1), 360.0 * da)) *
                    (hinv3 * hinv);
            dn[c] = fma(60.0 * h2, s1 - s0, fma(-360.0 * h, j0 + j1, 720.0 * da)) * (hinv3 * hinv2);
        }
    }
    if (!finite) atomicOr(flags, kFlagNonFinite);
    if (SHARED) return;
    // generalized Aarseth criterion, order 6: dt^6 = eta^6 A1 / A4
    const double A1 = fma(norm3(fa[0], fa[1], fa[2]), norm3(fs[0], fs[1], fs[2]),
                          fma(fj[0], fj[0], fma(fj[1], fj[1], fj[2] * fj[2])));
    const double A4 = fma(norm3(c1o[0], c1o[1], c1o[2]), norm3(dn[0], dn[1], dn[2]),
                          fma(pn[0], pn[0], fma(pn[1], pn[1], pn[2] * pn[2])));
    const double q = (A1 / A4) * eta6;
    const int lev_crit = level_from_power(q, 6, lev_min, lev_max + 1);
    const int lev_old = level_of_ticks(dt_old);
    int lev_new = lev_old;
    if (lev_crit > lev_old) {
        lev_new = lev_crit;
    } else if (lev_crit < lev_old) {
        const int64_t two_old = dt_old << 1;  // a power of two
        if ((t_next & (two_old - 1)) == 0) lev_new = lev_old - 1;
    }
    if (lev_new > lev_max) {
        atomicOr(flags, kFlagDtMin);
        lev_new = lev_max;
    }
    *lev_out = lev_new;
}

// correct_from with the old state read from st.
template <bool SHARED>
__device__ __forceinline__ void correct_vals(const h6_state &st, int i, const double *fa,
                                             const double *fj, const double *fs, int64_t t_next,
                                             double dt_sh, double eta6, int lev_min, int lev_max,
                                             int32_t *flags, double *x1o, double *v1o,
                                             double *c1o, int *lev_out) {
    correct_from<SHARED>(load_old<SHARED>(st, i), fa, fj, fs, t_next, dt_sh, eta6, lev_min,
                         lev_max, flags, x1o, v1o, c1o, lev_out);
}

// correct_vals, stored in place: x, v, c corrected, a, j, s the new
// values; block steps also set t = t_next and the new step.
template <bool SHARED>
__device__ __forceinline__ void correct_one(const h6_state &st, int i, const double *fa,
                                            const double *fj, const double *fs, int64_t t_next,
                                            double dt_sh, double eta6, int lev_min, int lev_max,
                                            int32_t *flags) {
    double x1[3], v1[3], c1[3];
    int lev = 0;
    correct_vals<SHARED>(st, i, fa, fj, fs, t_next, dt_sh, eta6, lev_min, lev_max, flags, x1, v1,
                         c1, &lev);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        st.x[c][i] = x1[c];
        st.v[c][i] = v1[c];
        st.a[c][i] = fa[c];
        st.j[c][i] = fj[c];
        st.s[c][i] = fs[c];
        st.c[c][i] = c1[c];
    }
    if (SHARED) return;
    st.t[i] = t_next;
    st.dt[i] = (int64_t)1 << (kTickBits - lev);
}

}  // namespace stepbody
}  // namespace h6
