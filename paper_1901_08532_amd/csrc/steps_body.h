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
// Taylor prediction of particle i over interval d: x to 5th order, v to
// 4th, a to 3rd, Horner form.
__device__ __forceinline__ void predict_one(const h6_state &st, int i, double d,
                                            const h6_pred &out) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double x = st.x[c][i], v = st.v[c][i], a = st.a[c][i];
        const double j = st.j[c][i], s = st.s[c][i], cr = st.c[c][i];
        // a_p = a + d (j + d/2 (s + d/3 c))
        const double ap = fma(d, fma(d * 0.5, fma(d * (1.0 / 3.0), cr, s), j), a);
        // v_p = v + d (a + d/2 (j + d/3 (s + d/4 c)))
        const double vp =
            fma(d, fma(d * 0.5, fma(d * (1.0 / 3.0), fma(d * 0.25, cr, s), j), a), v);
        // x_p = x + d (v + d/2 (a + d/3 (j + d/4 (s + d/5 c))))
        const double xp = fma(
            d, fma(d * 0.5, fma(d * (1.0 / 3.0), fma(d * 0.25, fma(d * 0.2, cr, s), j), a), v), x);
        out.x[c][i] = xp;
        out.v[c][i] = vp;
        out.a[c][i] = ap;
    }
}

// ---------------------------------------------------------------- corrector
// 6th-order Hermite corrector, quintic interpolation of crackle, pop and
// the fifth derivative at the step end, and the power-of-two step rule.
// Corrects particle i (k: its index in the force arrays) with the new
// a1, j1, s1 (fa, fj, fs); shared steps use the fixed step dt_sh and keep
// t and dt, block steps take the step from dt[i] and assign the new one.
template <bool SHARED>
__device__ __forceinline__ void correct_one(const h6_state &st, int i, const double *fa,
                                            const double *fj, const double *fs, int64_t t_next,
                                            double dt_sh, double eta6, int lev_min, int lev_max,
                                            int32_t *flags) {
    const int64_t dt_old = SHARED ? 0 : st.dt[i];
    const double h = SHARED ? dt_sh : (double)dt_old * kTick;
    const double h2 = h * h;
    const double hinv = 1.0 / h;
    const double hinv2 = hinv * hinv, hinv3 = hinv2 * hinv;
    double a1n[3], j1n[3], s1n[3], cn[3], pn[3], dn[3];
    bool finite = true;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double x0 = st.x[c][i], v0 = st.v[c][i];
        const double a0 = st.a[c][i], j0 = st.j[c][i], s0 = st.s[c][i];
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
        st.x[c][i] = x1;
        st.v[c][i] = v1;
        st.a[c][i] = a1;
        st.j[c][i] = j1;
        st.s[c][i] = s1;
        st.c[c][i] = c1;
        finite = finite && isfinite(x1) && isfinite(v1) && isfinite(c1);
        if (!SHARED) {
            const double p1 =
                fma(h2, 36.0 * s1 - 24.0 * s0, fma(-h, fma(168.0, j0, 192.0 * j1), 360.0 * da)) *
                (hinv3 * hinv);
            const double d5 =
                fma(60.0 * h2, s1 - s0, fma(-360.0 * h, j0 + j1, 720.0 * da)) * (hinv3 * hinv2);
            a1n[c] = a1;
            j1n[c] = j1;
            s1n[c] = s1;
            cn[c] = c1;
            pn[c] = p1;
            dn[c] = d5;
        }
    }
    if (!finite) atomicOr(flags, kFlagNonFinite);
    if (SHARED) return;
    // generalized Aarseth criterion, order 6: dt^6 = eta^6 A1 / A4
    const double A1 = fma(norm3(a1n[0], a1n[1], a1n[2]), norm3(s1n[0], s1n[1], s1n[2]),
                          fma(j1n[0], j1n[0], fma(j1n[1], j1n[1], j1n[2] * j1n[2])));
    const double A4 = fma(norm3(cn[0], cn[1], cn[2]), norm3(dn[0], dn[1], dn[2]),
                          fma(pn[0], pn[0], fma(pn[1], pn[1], pn[2] * pn[2])));
    const double q = (A1 / A4) * eta6;
    const int lev_crit = level_from_power(q, 6, lev_min, lev_max + 1);
    const int lev_old = level_of_ticks(dt_old);
    int lev_new = lev_old;
    if (lev_crit > lev_old) {
        lev_new = lev_crit;
    } else if (lev_crit < lev_old) {
        const int64_t two_old = dt_old << 1;
        if (t_next % two_old == 0) lev_new = lev_old - 1;
    }
    if (lev_new > lev_max) {
        atomicOr(flags, kFlagDtMin);
        lev_new = lev_max;
    }
    st.t[i] = t_next;
    st.dt[i] = (int64_t)1 << (kTickBits - lev_new);
}

}  // namespace stepbody
}  // namespace h6
