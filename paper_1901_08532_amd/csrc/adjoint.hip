// Adjoint of the shared-step Hermite-6 path: vector-Jacobian products of
// the a/j/s evaluation (and of the start-up passes), and the transposes of
// the shared-step predictor and corrector.
//
// Pair VJP. Write the sum on target k as F_k = sum_j m_j Q(r, v, a, jr)
// with r = x_j - x_k, v = v_j - v_k, a = a_j - a_k, jr = j_j - j_k and Q the
// pair terms per unit source mass (A, J, S or S, C). Q is odd in the joint
// argument, so its Jacobian is even, and the contributions of k as target
// and as source combine into one gather over the same pairs as the forward
// sum: with cotangents g of the outputs,
//   xbar_k = sum_j (dQ/dr)^T (m_k g_j - m_j g_k)      (likewise v, a, jr)
//   mbar_k = -sum_j Q . g_j.
// (dQ/d.)^T is applied by the hand reversal of the forward pair code:
// the forward values of R^-3, alpha, beta, gamma, w, u, z are recomputed,
// then their adjoints are accumulated in reverse order. The self pair
// (whose terms cancel in exact arithmetic) is excluded explicitly.
//
// Launch structure as the forward kernel: LDS tiles of source records,
// one target per lane, source slices combined by the compensated slice
// reduction; no floating-point atomics.
#include <algorithm>
#include <type_traits>

#include "device_math.h"
#include "h6_internal.h"

namespace h6 {
namespace {

template <int ORDER>
struct VTraits;
template <>  // start-up pass 1: outputs A, J; inputs x, v
struct VTraits<1> {
    static constexpr int NG = 6;    // output cotangent components
    static constexpr int NOUT = 7;  // xbar 3, vbar 3, mbar
    static constexpr int NF = 13;   // source record: x 3, v 3, m, g 6
};
template <>  // per step: outputs A, J, S; inputs x, v, a
struct VTraits<2> {
    static constexpr int NG = 9;
    static constexpr int NOUT = 10;  // xbar, vbar, abar, mbar
    static constexpr int NF = 19;    // x, v, a, m, g 9
};
template <>  // start-up pass 2: outputs S, C; inputs x, v, a, j
struct VTraits<3> {
    static constexpr int NG = 6;
    static constexpr int NOUT = 13;  // xbar, vbar, abar, jbar, mbar
    static constexpr int NF = 19;    // x, v, a, j, m, g 6
};

__device__ __forceinline__ double dot3(const double *p, const double *q) {
    return fma(p[2], q[2], fma(p[1], q[1], p[0] * q[0]));
}

// Reverse-mode pair: accumulates (dQ/dr)^T gh into xb, (dQ/dv)^T gh into vb,
// (dQ/da)^T gh into ab, (dQ/djr)^T gh into jb, and (MASS) -Q . gj into mb.
template <int ORDER, bool MASS = true>
__device__ __forceinline__ void pair_vjp(const double *r, const double *v, const double *a,
                                         const double *jr, double r2, const double *gh,
                                         const double *gj, double *xb, double *vb, double *ab,
                                         double *jb, double &mb) {
    // ---- forward values
    const double rho = rsqrt_f64(r2);
    const double rho2 = rho * rho;
    const double q3 = rho * rho2;  // R^-3
    const double rv = dot3(r, v);
    const double alpha = rv * rho2;
    double w[3], u[3] = {0, 0, 0}, z[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c) w[c] = fma(-3.0 * alpha, r[c], v[c]);
    double vvra = 0, beta = 0, va = 0, rj = 0, gamma = 0;
    if constexpr (ORDER >= 2) {
        vvra = fma(v[2], v[2], fma(v[1], v[1], v[0] * v[0])) + dot3(r, a);
        beta = fma(alpha, alpha, vvra * rho2);
#pragma unroll
        for (int c = 0; c < 3; ++c) u[c] = fma(-6.0 * alpha, w[c], fma(-3.0 * beta, r[c], a[c]));
    }
    if constexpr (ORDER == 3) {
        va = dot3(v, a);
        rj = dot3(r, jr);
        gamma = fma(alpha, fma(-4.0 * alpha, alpha, 3.0 * beta), fma(3.0, va, rj) * rho2);
#pragma unroll
        for (int c = 0; c < 3; ++c)
            z[c] = fma(-9.0 * alpha, u[c], fma(-9.0 * beta, w[c], fma(-3.0 * gamma, r[c], jr[c])));
    }
    // ---- cotangent layout of the outputs
    const double zero3[3] = {0, 0, 0};
    const double *Ab = ORDER == 3 ? zero3 : gh;
    const double *Jb = ORDER == 3 ? zero3 : gh + 3;
    const double *Sb = ORDER == 2 ? gh + 6 : ORDER == 3 ? gh : zero3;
    const double *Cb = ORDER == 3 ? gh + 3 : zero3;
    const double *Aj = ORDER == 3 ? zero3 : gj;
    const double *Jj = ORDER == 3 ? zero3 : gj + 3;
    const double *Sj = ORDER == 2 ? gj + 6 : ORDER == 3 ? gj : zero3;
    const double *Cj = ORDER == 3 ? gj + 3 : zero3;
    // mass: -Q . g_j with Q = R^-3 (r, w, u, z) for (A, J, S, C)
    if constexpr (MASS) {
        double qg = dot3(r, Aj) + dot3(w, Jj);
        if constexpr (ORDER >= 2) qg += dot3(u, Sj);
        if constexpr (ORDER == 3) qg += dot3(z, Cj);
        mb = fma(-q3, qg, mb);
    }
    // ---- reverse sweep
    double q3b = dot3(Ab, r) + dot3(Jb, w);
    if constexpr (ORDER >= 2) q3b += dot3(Sb, u);
    if constexpr (ORDER == 3) q3b += dot3(Cb, z);
    double rb[3], wb[3], ub[3], vbl[3] = {0, 0, 0}, abl[3] = {0, 0, 0}, jrb[3] = {0, 0, 0};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        rb[c] = q3 * Ab[c];
        wb[c] = q3 * Jb[c];
        ub[c] = q3 * Sb[c];
    }
    double alphab = 0, betab = 0, rho2b = 0;
    if constexpr (ORDER == 3) {
        double zb[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) zb[c] = q3 * Cb[c];
        // z = jr - 9 alpha u - 9 beta w - 3 gamma r
        const double gammab = -3.0 * dot3(r, zb);
        alphab = -9.0 * dot3(u, zb);
        betab = -9.0 * dot3(w, zb);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            jrb[c] = zb[c];
            ub[c] = fma(-9.0 * alpha, zb[c], ub[c]);
            wb[c] = fma(-9.0 * beta, zb[c], wb[c]);
            rb[c] = fma(-3.0 * gamma, zb[c], rb[c]);
        }
        // gamma = (3 v.a + r.jr) rho2 + alpha (3 beta - 4 alpha^2)
        const double gr = gammab * rho2;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            vbl[c] = fma(3.0 * gr, a[c], vbl[c]);
            abl[c] = fma(3.0 * gr, v[c], abl[c]);
            rb[c] = fma(gr, jr[c], rb[c]);
            jrb[c] = fma(gr, r[c], jrb[c]);
        }
        rho2b = gammab * fma(3.0, va, rj);
        alphab = fma(gammab, fma(-12.0 * alpha, alpha, 3.0 * beta), alphab);
        betab = fma(3.0 * alpha, gammab, betab);
    }
    if constexpr (ORDER >= 2) {
        // u = a - 6 alpha w - 3 beta r
        alphab = fma(-6.0, dot3(w, ub), alphab);
        betab = fma(-3.0, dot3(r, ub), betab);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            abl[c] += ub[c];
            wb[c] = fma(-6.0 * alpha, ub[c], wb[c]);
            rb[c] = fma(-3.0 * beta, ub[c], rb[c]);
        }
        // beta = (v.v + r.a) rho2 + alpha^2
        const double br = betab * rho2;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            vbl[c] = fma(2.0 * br, v[c], vbl[c]);
            rb[c] = fma(br, a[c], rb[c]);
            abl[c] = fma(br, r[c], abl[c]);
        }
        rho2b = fma(betab, vvra, rho2b);
        alphab = fma(2.0 * alpha, betab, alphab);
    }
    // w = v - 3 alpha r
    alphab = fma(-3.0, dot3(r, wb), alphab);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        vbl[c] += wb[c];
        rb[c] = fma(-3.0 * alpha, wb[c], rb[c]);
    }
    // alpha = (r.v) rho2
    const double ar = alphab * rho2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        rb[c] = fma(ar, v[c], rb[c]);
        vbl[c] = fma(ar, r[c], vbl[c]);
    }
    rho2b = fma(alphab, rv, rho2b);
    // q3 = R2^(-3/2), rho2 = R2^(-1), R2 = r.r + eps^2
    const double r2b = -1.5 * q3b * q3 * rho2 - rho2b * rho2 * rho2;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xb[c] += fma(2.0 * r2b, r[c], rb[c]);
        vb[c] += vbl[c];
        if constexpr (ORDER >= 2) ab[c] += abl[c];
        if constexpr (ORDER == 3) jb[c] += jrb[c];
    }
}

struct CotPtrs {
    const double *g[9];
};

constexpr double kPadPosVjp = 1.0e18;

// Which pairs and which half of each pair a launch covers. With the
// cotangents g nonzero only on an active set (block steps), the pair sum
// splits into a source half m_k g_j over the active sources j, for every
// target k (with the mass term), and a target half -m_j g_k over all
// sources, for the active targets k: 2 n_act n pairs instead of n^2.
//   kAll:        targets 0..n-1 against sources 0..n-1, both halves;
//   kSrcHalf:    targets 0..n-1 against the sources list[0..n_list),
//                their cotangents given by list rank;
//   kTargetHalf: targets list[0..n_list) (cotangents by rank) against
//                sources 0..n-1; outputs by rank, without the mass term.
// Every mode skips the self pair.
enum VjpMode { kAll = 0, kSrcHalf = 1, kTargetHalf = 2 };

// Order-2 pair VJP, factored. With gh = m_k g_j - m_j g_k and
//   G(g)  = gA.r + gJ.w + gS.u
//         = gA.r + gJ.v - 3 alpha gJ.r + gS.a - 6 alpha gS.v + c18 gS.r,
//   c18   = 18 alpha^2 - 3 beta,
//   Ga(g) = -3 gJ.r - 6 gS.v + 30 alpha gS.r    (dG/dalpha, beta's alpha^2
//                                                included),
// the pair's contribution Q . gh = R^-3 G(gh) has the gradients
//   d/dr: R^-3 (gA - 3 alpha gJ + c18 gS) + sa v + sb a + cr r,
//   d/dv: R^-3 (gJ - 6 alpha gS) + sa r + 2 sb v,
//   d/da: R^-3 gS + sb r,
// with sa = R^-5 Ga(gh), sb = -3 R^-5 gS.r, cr = -3 R^-5 G(gh) - 2 alpha sa
// - 2 beta' sb, beta' = (v.v + r.a)/R^2. G, Ga and gS.r are linear in g, so
// they come from six dot products with each of g_j and g_k; the explicit
// terms of the target's own cotangent, -m_j R^-3 (...)(g_k), are
// accumulated as three scalar sums (sum m_j R^-3, alpha m_j R^-3,
// c18 m_j R^-3) and applied to g_k once per slice. MODE drops the g_j
// part (kTargetHalf) or the g_k part (kSrcHalf); the mass term -R^-3 G(g_j)
// goes with the g_j part.
__device__ __forceinline__ void g_terms(const double *g, const double *r, const double *v,
                                        const double *a, double a3, double a6, double c18,
                                        double a30, double &G, double &Ga, double &dSr) {
    const double dAr = dot3(g, r), dJr = dot3(g + 3, r), dJv = dot3(g + 3, v);
    dSr = dot3(g + 6, r);
    const double dSv = dot3(g + 6, v), dSa = dot3(g + 6, a);
    G = fma(c18, dSr, fma(-a6, dSv, fma(-a3, dJr, dAr + dJv) + dSa));
    Ga = fma(a30, dSr, fma(-6.0, dSv, -3.0 * dJr));
}

template <int MODE>
__device__ __forceinline__ void pair_vjp2(const double *r, const double *v, const double *a,
                                          double r2, double mk, double mj, const double *gj,
                                          const double *gk, double *acc, double *sacc) {
    constexpr bool GJ = MODE != kTargetHalf, GK = MODE != kSrcHalf;
    const double rho = rsqrt_f64(r2);
    const double rho2 = rho * rho;
    const double q3 = rho * rho2;
    const double alpha = dot3(r, v) * rho2;
    const double bp = (fma(v[2], v[2], fma(v[1], v[1], v[0] * v[0])) + dot3(r, a)) * rho2;
    const double beta = fma(alpha, alpha, bp);
    const double a3 = 3.0 * alpha;
    const double a6 = a3 + a3;
    const double c18 = fma(6.0 * a3, alpha, -3.0 * beta);
    const double a30 = 10.0 * a3;
    double G = 0.0, Ga = 0.0, dS = 0.0, Gj = 0.0;
    if constexpr (GJ) {
        double Gaj, dSj;
        g_terms(gj, r, v, a, a3, a6, c18, a30, Gj, Gaj, dSj);
        G = mk * Gj;
        Ga = mk * Gaj;
        dS = mk * dSj;
    }
    if constexpr (GK) {
        double Gk, Gak, dSk;
        g_terms(gk, r, v, a, a3, a6, c18, a30, Gk, Gak, dSk);
        G = fma(-mj, Gk, G);
        Ga = fma(-mj, Gak, Ga);
        dS = fma(-mj, dSk, dS);
    }
    const double qr = q3 * rho2;
    const double sa = qr * Ga;
    const double sb = (-3.0 * qr) * dS;
    const double cr = fma(-3.0 * qr, G, fma(-2.0 * alpha, sa, (-2.0 * bp) * sb));
    const double sb2 = sb + sb;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc[c] = fma(sa, v[c], fma(sb, a[c], fma(cr, r[c], acc[c])));
        acc[3 + c] = fma(sa, r[c], fma(sb2, v[c], acc[3 + c]));
        acc[6 + c] = fma(sb, r[c], acc[6 + c]);
    }
    if constexpr (GJ) {
        const double kq = mk * q3;
        const double kqa = -a3 * kq, kqc = c18 * kq;
        const double kqa6 = kqa + kqa;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            acc[c] = fma(kq, gj[c], fma(kqa, gj[3 + c], fma(kqc, gj[6 + c], acc[c])));
            acc[3 + c] = fma(kq, gj[3 + c], fma(kqa6, gj[6 + c], acc[3 + c]));
            acc[6 + c] = fma(kq, gj[6 + c], acc[6 + c]);
        }
        acc[9] = fma(-q3, Gj, acc[9]);
    }
    if constexpr (GK) {
        const double jq = mj * q3;
        sacc[0] += jq;
        sacc[1] = fma(jq, alpha, sacc[1]);
        sacc[2] = fma(jq, c18, sacc[2]);
    }
}

template <int ORDER, int BLOCK, int MODE = kAll>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2))) void k_eval_vjp(
    SrcPtrs src, CotPtrs cot, int n, const int32_t *__restrict__ list, int n_list, double eps2,
    int slice_len, OutPtrs out, int64_t slice_stride, unsigned acc_mask) {
    using T = VTraits<ORDER>;
    constexpr int NG = T::NG, NOUT = T::NOUT, NF = T::NF;
    constexpr int NFP = (NF + 1) & ~1;  // record padded to whole double2
    constexpr bool MASS = MODE != kTargetHalf;
    constexpr bool SKIP = MODE != kAll;  // the list modes identify the self pair by particle
    __shared__ double2 tile[BLOCK * NFP / 2];
    const int tid = threadIdx.x;
    const int k = (int)blockIdx.x * BLOCK + tid;
    const int n_tgt = MODE == kTargetHalf ? n_list : n;
    const int n_src = MODE == kSrcHalf ? n_list : n;
    const int kr = k < n_tgt ? k : n_tgt - 1;                  // target rank
    const int kc = MODE == kTargetHalf ? list[kr] : kr;        // target particle

    double xk[3], vk[3], ak[3] = {0, 0, 0}, jk[3] = {0, 0, 0}, gk[NG];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xk[c] = src.x[c][kc];
        vk[c] = src.v[c][kc];
        if constexpr (ORDER >= 2) ak[c] = src.a[c][kc];
        if constexpr (ORDER == 3) jk[c] = src.j[c][kc];
    }
    const double mk = src.m[kc];
#pragma unroll
    for (int q = 0; q < NG; ++q) gk[q] = MODE == kSrcHalf ? 0.0 : cot.g[q][kr];

    double acc[NOUT], hi[NOUT], lo[NOUT];
#pragma unroll
    for (int q = 0; q < NOUT; ++q) acc[q] = hi[q] = lo[q] = 0.0;
    // order 2: scalar sums for the target's own cotangent (pair_vjp2)
    constexpr bool SK = ORDER == 2 && MODE != kSrcHalf;
    double sacc[3] = {0, 0, 0}, shi[3] = {0, 0, 0}, slo[3] = {0, 0, 0};

    const int jb0 = (int)blockIdx.y * slice_len;
    const int je = min(n_src, jb0 + slice_len);
    __shared__ int tile_id[BLOCK];  // source particle of each record (self test)
    for (int jt = jb0; jt < je; jt += BLOCK) {
        __syncthreads();
        {
            double f[NFP];
            const int jj = jt + tid;  // source rank
            if (jj < je) {
                const int pj = MODE == kSrcHalf ? list[jj] : jj;
                if constexpr (SKIP) tile_id[tid] = pj;
                int o = 0;
#pragma unroll
                for (int c = 0; c < 3; ++c) f[o++] = src.x[c][pj];
#pragma unroll
                for (int c = 0; c < 3; ++c) f[o++] = src.v[c][pj];
                if constexpr (ORDER >= 2) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) f[o++] = src.a[c][pj];
                }
                if constexpr (ORDER == 3) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) f[o++] = src.j[c][pj];
                }
                f[o++] = src.m[pj];
#pragma unroll
                for (int q = 0; q < NG; ++q) f[o++] = MODE == kTargetHalf ? 0.0 : cot.g[q][jj];
            } else {
                if constexpr (SKIP) tile_id[tid] = -1;
#pragma unroll
                for (int q = 0; q < NFP; ++q) f[q] = 0.0;
                f[0] = f[1] = f[2] = kPadPosVjp;  // far and massless, zero cotangent
            }
            if (NFP > NF) f[NFP - 1] = 0.0;
#pragma unroll
            for (int q = 0; q < NFP / 2; ++q) tile[tid * (NFP / 2) + q] = make_double2(f[2 * q], f[2 * q + 1]);
        }
        __syncthreads();
        auto tile_pairs = [&](auto test_self) {
            for (int q = 0; q < BLOCK; ++q) {
                double f[NFP];
#pragma unroll
                for (int p = 0; p < NFP / 2; ++p) {
                    const double2 d = tile[q * (NFP / 2) + p];
                    f[2 * p] = d.x;
                    f[2 * p + 1] = d.y;
                }
                int o = 0;
                double r[3], v[3], a[3] = {0, 0, 0}, jr[3] = {0, 0, 0};
#pragma unroll
                for (int c = 0; c < 3; ++c) r[c] = f[o++] - xk[c];
#pragma unroll
                for (int c = 0; c < 3; ++c) v[c] = f[o++] - vk[c];
                if constexpr (ORDER >= 2) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) a[c] = f[o++] - ak[c];
                }
                if constexpr (ORDER == 3) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) jr[c] = f[o++] - jk[c];
                }
                // The self pair is left out explicitly: m_k g_k - m_k g_k is not
                // exactly zero once the first product is fused (fma keeps its
                // rounding error), and dQ/dr at r = 0 is of order eps^-3. With
                // both masses set to zero gh is exactly zero; r, v, a, jr are zero
                // there, so Q and the mass term are too (R^2 set to 1 keeps them
                // finite when eps = 0).
                const bool self = decltype(test_self)::value &&
                                  (MODE == kAll ? (jt + q) == k : tile_id[q] == kc);
                const double mj = self ? 0.0 : f[o];
                const double mkp = self ? 0.0 : mk;
                ++o;
                const double *gj = &f[o];
                double r2 = fma(r[2], r[2], fma(r[1], r[1], fma(r[0], r[0], eps2)));
                r2 = self ? 1.0 : r2;
                if constexpr (ORDER == 2) {
                    pair_vjp2<MODE>(r, v, a, r2, mkp, mj, gj, gk, acc, sacc);
                } else {
                    double gh[NG];
#pragma unroll
                    for (int p = 0; p < NG; ++p) {
                        if constexpr (MODE == kAll) gh[p] = fma(mkp, gj[p], -mj * gk[p]);
                        else if constexpr (MODE == kSrcHalf) gh[p] = mkp * gj[p];
                        else gh[p] = -mj * gk[p];
                    }
                    double *xb = acc, *vb = acc + 3;
                    double *ab = ORDER >= 2 ? acc + 6 : acc;  // unused for order 1
                    double *jb = ORDER == 3 ? acc + 9 : acc;  // unused below order 3
                    pair_vjp<ORDER, MASS>(r, v, a, jr, r2, gh, gj, xb, vb, ab, jb, acc[NOUT - 1]);
                }
            }
        };
        // in the all-pairs mode a self pair can only occur in the diagonal
        // tile (slices are whole tiles aligned with the target blocks)
        if (MODE != kAll || jt == (int)blockIdx.x * BLOCK)
            tile_pairs(std::true_type{});
        else
            tile_pairs(std::false_type{});
#pragma unroll
        for (int q = 0; q < NOUT; ++q) {
            two_sum_into(hi[q], lo[q], acc[q]);
            acc[q] = 0.0;
        }
        if constexpr (SK) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                two_sum_into(shi[q], slo[q], sacc[q]);
                sacc[q] = 0.0;
            }
        }
    }
    if constexpr (SK) {
        // the target's own cotangent: -S0 gA + 3 S1 gJ - S2 gS into xbar,
        // -S0 gJ + 6 S1 gS into vbar, -S0 gS into abar
        const double S0 = shi[0] + slo[0], S1 = shi[1] + slo[1], S2 = shi[2] + slo[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            two_sum_into(hi[c], lo[c], fma(-S0, gk[c], fma(3.0 * S1, gk[3 + c], -S2 * gk[6 + c])));
            two_sum_into(hi[3 + c], lo[3 + c], fma(-S0, gk[3 + c], 6.0 * S1 * gk[6 + c]));
            two_sum_into(hi[6 + c], lo[6 + c], -S0 * gk[6 + c]);
        }
    }
    if (k < n_tgt) {
        const int64_t soff = (int64_t)blockIdx.y * slice_stride;
#pragma unroll
        for (int q = 0; q < (MASS ? NOUT : NOUT - 1); ++q) {
            double *dst = &out.p[q][soff + k];
            const double val = hi[q] + lo[q];
            *dst = ((acc_mask >> q) & 1u) ? *dst + val : val;
        }
    }
}

// Transpose of the shared-step corrector. Forward (step h, per component):
//   v1 = v + h/2 (a + A1) - h^2/10 (J1 - j) + h^3/120 (s + S1)
//   x1 = x + h/2 (v + v1) - h^2/10 (A1 - a) + h^3/120 (j + J1)
//   c1 = [60 (A1 - a) - h (24 j + 36 J1) + h^2 (9 S1 - 3 s)] / h^3
//   a1 = A1, j1 = J1, s1 = S1.
// In: cotangents of (x1, v1, a1, j1, s1, c1) in cot. Out: cotangents of the
// old (x, v, a, j, s) in cot (c's set to zero: the old crackle enters only
// the predictor), and of the evaluated (A1, J1, S1) in cf.
__global__ __launch_bounds__(256) void k_correct_shared_vjp(h6_state cot, int n, h6_force cf,
                                                            double h) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double h2 = h * h, h3 = h2 * h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double X = cot.x[c][i], V = cot.v[c][i], Ab = cot.a[c][i];
        const double Jb = cot.j[c][i], Sb = cot.s[c][i], Cb = cot.c[c][i];
        const double V1 = fma(0.5 * h, X, V);  // cotangent of v1 (x1 depends on it)
        const double xo = X;
        const double vo = fma(0.5 * h, X, V1);
        const double ao = fma(0.1 * h2, X, fma(0.5 * h, V1, -60.0 / h3 * Cb));
        const double jo = fma(h3 / 120.0, X, fma(0.1 * h2, V1, -24.0 / h2 * Cb));
        const double so = fma(h3 / 120.0, V1, -3.0 / h * Cb);
        const double A1 = Ab + fma(-0.1 * h2, X, fma(0.5 * h, V1, 60.0 / h3 * Cb));
        const double J1 = Jb + fma(h3 / 120.0, X, fma(-0.1 * h2, V1, -36.0 / h2 * Cb));
        const double S1 = Sb + fma(h3 / 120.0, V1, 9.0 / h * Cb);
        cot.x[c][i] = xo;
        cot.v[c][i] = vo;
        cot.a[c][i] = ao;
        cot.j[c][i] = jo;
        cot.s[c][i] = so;
        cot.c[c][i] = 0.0;
        cf.a[c][i] = A1;
        cf.j[c][i] = J1;
        cf.s[c][i] = S1;
    }
}

// Transpose of the shared-step predictor (Taylor series over h), added to
// the state cotangents:
//   xbar += xpb; vbar += h xpb + vpb; abar += h^2/2 xpb + h vpb + apb;
//   jbar += h^3/6 xpb + h^2/2 vpb + h apb; sbar += h^4/24 xpb + h^3/6 vpb
//   + h^2/2 apb; cbar += h^5/120 xpb + h^4/24 vpb + h^3/6 apb.
__global__ __launch_bounds__(256) void k_predict_dt_vjp(h6_state cot, int n, h6_pred cp, double h) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double X = cp.x[c][i], V = cp.v[c][i], A = cp.a[c][i];
        cot.x[c][i] += X;
        cot.v[c][i] += fma(h, X, V);
        cot.a[c][i] += fma(0.5 * h2, X, fma(h, V, A));
        cot.j[c][i] += fma(h3 / 6.0, X, fma(0.5 * h2, V, h * A));
        cot.s[c][i] += fma(h4 / 24.0, X, fma(h3 / 6.0, V, 0.5 * h2 * A));
        cot.c[c][i] += fma(h5 / 120.0, X, fma(h4 / 24.0, V, h3 / 6.0 * A));
    }
}

int ceil_div_i(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Sum of slice partials [slice][comp][rank] (ld = n_list) added to
// out.p[comp][list[rank]]: the target half's results scattered to the
// particles (list entries are distinct, so no two ranks meet).
__global__ __launch_bounds__(256) void k_reduce_scatter(const double *__restrict__ partial,
                                                        int64_t ld, int n_split, int ncomp,
                                                        const int32_t *__restrict__ list,
                                                        int n_list, OutPtrs out) {
    const int64_t total = (int64_t)ncomp * n_list;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int c = (int)(idx / n_list);
        const int k = (int)(idx - (int64_t)c * n_list);
        double hi = 0.0, lo = 0.0;
        for (int sl = 0; sl < n_split; ++sl)
            two_sum_into(hi, lo, partial[((int64_t)sl * ncomp + c) * ld + k]);
        out.p[c][list[k]] += hi + lo;
    }
}

template <int ORDER, int MODE>
hipError_t launch_vjp_mode(h6_ctx ctx, const SrcPtrs &src, const CotPtrs &cot, int n,
                           const int32_t *list, int n_list, const OutPtrs &out,
                           unsigned acc_mask) {
    constexpr int BLOCK = 128;
    constexpr int NOUT = VTraits<ORDER>::NOUT;
    constexpr int NW = MODE == kTargetHalf ? NOUT - 1 : NOUT;  // outputs written
    const int n_tgt = MODE == kTargetHalf ? n_list : n;
    const int n_src = MODE == kSrcHalf ? n_list : n;
    if (n_tgt <= 0 || n_src <= 0) return hipSuccess;
    const int blocks_i = ceil_div_i(n_tgt, BLOCK);
    int split = balanced_split(ctx, 2, BLOCK, n_src, blocks_i);
    const int64_t cap = ctx->partial_cap / ((int64_t)NW * n_tgt);
    if (split > cap) split = (int)std::max<int64_t>(1, cap);
    int slice_len = ceil_div_i(ceil_div_i(n_src, split), BLOCK) * BLOCK;
    split = ceil_div_i(n_src, slice_len);
    // the target half always goes through the partials (scattered after)
    const bool direct = split == 1 && MODE != kTargetHalf;
    OutPtrs dst;
    int64_t slice_stride = 0;
    unsigned mask = acc_mask;
    if (direct) {
        dst = out;
    } else {
        for (int c = 0; c < kMaxOut; ++c) dst.p[c] = nullptr;
        for (int c = 0; c < NW; ++c) dst.p[c] = ctx->partial + (int64_t)c * n_tgt;
        slice_stride = (int64_t)NW * n_tgt;
        mask = 0u;  // partials are overwritten; the reduction applies acc_mask
    }
    dim3 grid(blocks_i, split);
    hipLaunchKernelGGL((k_eval_vjp<ORDER, BLOCK, MODE>), grid, dim3(BLOCK), 0, ctx->stream, src,
                       cot, n, list, n_list, ctx->eps2, slice_len, dst, slice_stride, mask);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || direct) return e;
    if constexpr (MODE == kTargetHalf) {
        int rb = ceil_div_i((int64_t)NW * n_tgt, 256);
        if (rb > 4096) rb = 4096;
        hipLaunchKernelGGL(k_reduce_scatter, dim3(rb), dim3(256), 0, ctx->stream, ctx->partial,
                           (int64_t)n_tgt, split, NW, list, n_tgt, out);
        return hipGetLastError();
    } else {
        return launch_reduce(ctx, split, NOUT, 0, n_tgt, out, acc_mask);
    }
}

template <int ORDER>
hipError_t launch_vjp_order(h6_ctx ctx, const SrcPtrs &src, const CotPtrs &cot, int n,
                            const OutPtrs &out, unsigned acc_mask) {
    return launch_vjp_mode<ORDER, kAll>(ctx, src, cot, n, nullptr, 0, out, acc_mask);
}

// Transpose of the block-step corrector for the active particles, each over
// its own step (dt_old, ticks): the shared-step transpose with h per
// particle; cf by rank.
__global__ __launch_bounds__(256) void k_correct_block_vjp(h6_state cot,
                                                           const int32_t *__restrict__ active,
                                                           int n_act,
                                                           const int64_t *__restrict__ dt_old,
                                                           h6_force cf) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_act) return;
    const int i = active[k];
    const double h = (double)dt_old[i] * (1.0 / (double)((int64_t)1 << kTickBits));
    const double h2 = h * h, h3 = h2 * h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double X = cot.x[c][i], V = cot.v[c][i], Ab = cot.a[c][i];
        const double Jb = cot.j[c][i], Sb = cot.s[c][i], Cb = cot.c[c][i];
        const double V1 = fma(0.5 * h, X, V);
        cot.x[c][i] = X;
        cot.v[c][i] = fma(0.5 * h, X, V1);
        cot.a[c][i] = fma(0.1 * h2, X, fma(0.5 * h, V1, -60.0 / h3 * Cb));
        cot.j[c][i] = fma(h3 / 120.0, X, fma(0.1 * h2, V1, -24.0 / h2 * Cb));
        cot.s[c][i] = fma(h3 / 120.0, V1, -3.0 / h * Cb);
        cot.c[c][i] = 0.0;
        cf.a[c][k] = Ab + fma(-0.1 * h2, X, fma(0.5 * h, V1, 60.0 / h3 * Cb));
        cf.j[c][k] = Jb + fma(h3 / 120.0, X, fma(-0.1 * h2, V1, -36.0 / h2 * Cb));
        cf.s[c][k] = Sb + fma(h3 / 120.0, V1, 9.0 / h * Cb);
    }
}

// Transpose of the block-step predictor: the shared-step transpose with the
// interval of each particle, d = (t_tick - t_old[i]) ticks.
__global__ __launch_bounds__(256) void k_predict_block_vjp(h6_state cot, int n,
                                                           const int64_t *__restrict__ t_old,
                                                           int64_t t_tick, h6_pred cp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double h = (double)(t_tick - t_old[i]) * (1.0 / (double)((int64_t)1 << kTickBits));
    const double h2 = h * h, h3 = h2 * h, h4 = h3 * h, h5 = h4 * h;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double X = cp.x[c][i], V = cp.v[c][i], A = cp.a[c][i];
        cot.x[c][i] += X;
        cot.v[c][i] += fma(h, X, V);
        cot.a[c][i] += fma(0.5 * h2, X, fma(h, V, A));
        cot.j[c][i] += fma(h3 / 6.0, X, fma(0.5 * h2, V, h * A));
        cot.s[c][i] += fma(h4 / 24.0, X, fma(h3 / 6.0, V, 0.5 * h2 * A));
        cot.c[c][i] += fma(h5 / 120.0, X, fma(h4 / 24.0, V, h3 / 6.0 * A));
    }
}

// Potential of each particle, phi_i = -sum_{j != i} m_j / sqrt(r^2 + eps^2):
// one target per lane over LDS tiles of (x, m), compensated per tile.
constexpr int kPotBlock = 256;
__global__ __launch_bounds__(kPotBlock) void k_potential(h6_state st, int n, double eps2,
                                                         double *__restrict__ phi) {
    __shared__ double4 tile[kPotBlock];
    const int tid = threadIdx.x;
    const int i = (int)blockIdx.x * kPotBlock + tid;
    const int ic = i < n ? i : n - 1;
    const double xi = st.x[0][ic], yi = st.x[1][ic], zi = st.x[2][ic];
    double hi = 0.0, lo = 0.0;
    for (int jt = 0; jt < n; jt += kPotBlock) {
        __syncthreads();
        const int jj = jt + tid;
        tile[tid] = jj < n ? make_double4(st.x[0][jj], st.x[1][jj], st.x[2][jj], st.m[jj])
                           : make_double4(kPadPosVjp, kPadPosVjp, kPadPosVjp, 0.0);
        __syncthreads();
        double acc = 0.0;
        const int cnt = min(kPotBlock, n - jt);
        for (int q = 0; q < cnt; ++q) {
            const double4 t = tile[q];
            const double dx = t.x - xi, dy = t.y - yi, dz = t.z - zi;
            const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
            const bool self = jt + q == ic;
            acc = fma(self ? 0.0 : t.w, rsqrt_f64(self ? 1.0 : r2), acc);
        }
        two_sum_into(hi, lo, acc);
    }
    if (i < n) phi[i] = -(hi + lo);
}

// Gradient of the total energy E = sum_i m_i |v_i|^2 / 2 - sum_{i<j} m_i m_j
// (r_ij^2 + eps^2)^(-1/2) scaled by its cotangent g (one device double; NULL:
// 1): dE/dx_i = -m_i a_i with a_i the softened acceleration, dE/dv_i =
// m_i v_i, dE/dm_i = |v_i|^2 / 2 + phi_i with phi_i the potential. One target
// per lane over LDS tiles of (x, m); phi and a share each pair's r^2 and
// 1/sqrt, compensated per tile.
__global__ __launch_bounds__(kPotBlock) void k_energy_vjp(h6_state st, int n, double eps2,
                                                          const double *__restrict__ cot,
                                                          h6_state out) {
    __shared__ double4 tile[kPotBlock];
    const int tid = threadIdx.x;
    const int i = (int)blockIdx.x * kPotBlock + tid;
    const int ic = i < n ? i : n - 1;
    const double xi = st.x[0][ic], yi = st.x[1][ic], zi = st.x[2][ic];
    double hi[4] = {0.0, 0.0, 0.0, 0.0}, lo[4] = {0.0, 0.0, 0.0, 0.0};  // phi, a
    for (int jt = 0; jt < n; jt += kPotBlock) {
        __syncthreads();
        const int jj = jt + tid;
        tile[tid] = jj < n ? make_double4(st.x[0][jj], st.x[1][jj], st.x[2][jj], st.m[jj])
                           : make_double4(kPadPosVjp, kPadPosVjp, kPadPosVjp, 0.0);
        __syncthreads();
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        const int cnt = min(kPotBlock, n - jt);
        for (int q = 0; q < cnt; ++q) {
            const double4 t = tile[q];
            const double dx = t.x - xi, dy = t.y - yi, dz = t.z - zi;
            const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
            const bool self = jt + q == ic;
            const double rinv = rsqrt_f64(self ? 1.0 : r2);
            const double mr = (self ? 0.0 : t.w) * rinv;
            const double mr3 = mr * (rinv * rinv);
            acc[0] += mr;
            acc[1] = fma(mr3, dx, acc[1]);
            acc[2] = fma(mr3, dy, acc[2]);
            acc[3] = fma(mr3, dz, acc[3]);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) two_sum_into(hi[q], lo[q], acc[q]);
    }
    if (i >= n) return;
    const double g = cot ? *cot : 1.0;
    const double mi = st.m[i];
    double vv = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double vc = st.v[c][i];
        vv = fma(vc, vc, vv);
        out.x[c][i] = -g * (mi * (hi[1 + c] + lo[1 + c]));
        out.v[c][i] = g * (mi * vc);
    }
    out.m[i] = g * fma(0.5, vv, -(hi[0] + lo[0]));
}

}  // namespace

hipError_t launch_energy_vjp(h6_ctx ctx, const h6_state *st, int n, const double *cot,
                             h6_state *out) {
    hipLaunchKernelGGL(k_energy_vjp, dim3((n + kPotBlock - 1) / kPotBlock), dim3(kPotBlock), 0,
                       ctx->stream, *st, n, ctx->eps2, cot, *out);
    return hipGetLastError();
}

hipError_t launch_eval_vjp(h6_ctx ctx, int order, const SrcPtrs &src, const double *const *cot,
                           int n, const OutPtrs &out, unsigned acc_mask) {
    CotPtrs cp;
    const int ng = order == 2 ? 9 : 6;
    for (int q = 0; q < 9; ++q) cp.g[q] = q < ng ? cot[q] : nullptr;
    if (order == 1) return launch_vjp_order<1>(ctx, src, cp, n, out, acc_mask);
    if (order == 2) return launch_vjp_order<2>(ctx, src, cp, n, out, acc_mask);
    return launch_vjp_order<3>(ctx, src, cp, n, out, acc_mask);
}

hipError_t launch_correct_shared_vjp(h6_ctx ctx, h6_state *cot, int n, const h6_force *cf,
                                     double dt) {
    hipLaunchKernelGGL(k_correct_shared_vjp, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, *cot,
                       n, *cf, dt);
    return hipGetLastError();
}

hipError_t launch_predict_dt_vjp(h6_ctx ctx, h6_state *cot, int n, const h6_pred *cp, double dt) {
    hipLaunchKernelGGL(k_predict_dt_vjp, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, *cot, n,
                       *cp, dt);
    return hipGetLastError();
}

hipError_t launch_eval_vjp_active(h6_ctx ctx, const SrcPtrs &src, const double *const *cot, int n,
                                  const int32_t *active, int n_act, const OutPtrs &out) {
    CotPtrs cp;
    for (int q = 0; q < 9; ++q) cp.g[q] = cot[q];
    // source half with the mass term, added to all ten outputs
    hipError_t e = launch_vjp_mode<2, kSrcHalf>(ctx, src, cp, n, active, n_act, out, 0x3ffu);
    if (e != hipSuccess) return e;
    // target half, scattered (added) to the active particles
    return launch_vjp_mode<2, kTargetHalf>(ctx, src, cp, n, active, n_act, out, 0x3ffu);
}

hipError_t launch_correct_block_vjp(h6_ctx ctx, h6_state *cot, const int32_t *active, int n_act,
                                    const int64_t *dt_old, const h6_force *cf) {
    if (n_act <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_correct_block_vjp, dim3((n_act + 255) / 256), dim3(256), 0, ctx->stream,
                       *cot, active, n_act, dt_old, *cf);
    return hipGetLastError();
}

hipError_t launch_predict_block_vjp(h6_ctx ctx, h6_state *cot, int n, const int64_t *t_old,
                                    int64_t t_tick, const h6_pred *cp) {
    hipLaunchKernelGGL(k_predict_block_vjp, dim3((n + 255) / 256), dim3(256), 0, ctx->stream,
                       *cot, n, t_old, t_tick, *cp);
    return hipGetLastError();
}

hipError_t launch_potential(h6_ctx ctx, const h6_state *st, int n, double *phi) {
    hipLaunchKernelGGL(k_potential, dim3((n + kPotBlock - 1) / kPotBlock), dim3(kPotBlock), 0,
                       ctx->stream, *st, n, ctx->eps2, phi);
    return hipGetLastError();
}

}  // namespace h6
