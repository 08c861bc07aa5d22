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
// then their adjoints are accumulated in reverse order. The self pair has
// m_k g_k - m_k g_k = 0 and Q = 0, so it contributes nothing.
//
// Launch structure as the forward kernel: LDS tiles of source records,
// one target per lane, source slices combined by the compensated slice
// reduction; no floating-point atomics.
#include <algorithm>

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
// (dQ/da)^T gh into ab, (dQ/djr)^T gh into jb, and -Q . gj into mb.
template <int ORDER>
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
    double qg = dot3(r, Aj) + dot3(w, Jj);
    if constexpr (ORDER >= 2) qg += dot3(u, Sj);
    if constexpr (ORDER == 3) qg += dot3(z, Cj);
    mb = fma(-q3, qg, mb);
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

template <int ORDER, int BLOCK, bool SKIPSELF>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(2))) void k_eval_vjp(
    SrcPtrs src, CotPtrs cot, int n, double eps2, int slice_len, OutPtrs out,
    int64_t slice_stride, unsigned acc_mask) {
    using T = VTraits<ORDER>;
    constexpr int NG = T::NG, NOUT = T::NOUT, NF = T::NF;
    constexpr int NFP = (NF + 1) & ~1;  // record padded to whole double2
    __shared__ double2 tile[BLOCK * NFP / 2];
    const int tid = threadIdx.x;
    const int k = (int)blockIdx.x * BLOCK + tid;
    const int kc = k < n ? k : n - 1;

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
    for (int q = 0; q < NG; ++q) gk[q] = cot.g[q][kc];

    double acc[NOUT], hi[NOUT], lo[NOUT];
#pragma unroll
    for (int q = 0; q < NOUT; ++q) acc[q] = hi[q] = lo[q] = 0.0;

    const int jb0 = (int)blockIdx.y * slice_len;
    const int je = min(n, jb0 + slice_len);
    for (int jt = jb0; jt < je; jt += BLOCK) {
        __syncthreads();
        {
            double f[NFP];
            const int jj = jt + tid;
            if (jj < je) {
                int o = 0;
#pragma unroll
                for (int c = 0; c < 3; ++c) f[o++] = src.x[c][jj];
#pragma unroll
                for (int c = 0; c < 3; ++c) f[o++] = src.v[c][jj];
                if constexpr (ORDER >= 2) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) f[o++] = src.a[c][jj];
                }
                if constexpr (ORDER == 3) {
#pragma unroll
                    for (int c = 0; c < 3; ++c) f[o++] = src.j[c][jj];
                }
                f[o++] = src.m[jj];
#pragma unroll
                for (int q = 0; q < NG; ++q) f[o++] = cot.g[q][jj];
            } else {
#pragma unroll
                for (int q = 0; q < NFP; ++q) f[q] = 0.0;
                f[0] = f[1] = f[2] = kPadPosVjp;  // far and massless, zero cotangent
            }
            if (NFP > NF) f[NFP - 1] = 0.0;
#pragma unroll
            for (int q = 0; q < NFP / 2; ++q) tile[tid * (NFP / 2) + q] = make_double2(f[2 * q], f[2 * q + 1]);
        }
        __syncthreads();
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
            const double mj = f[o++];
            const double *gj = &f[o];
            double gh[NG];
#pragma unroll
            for (int p = 0; p < NG; ++p) gh[p] = fma(mk, gj[p], -mj * gk[p]);
            double r2 = fma(r[2], r[2], fma(r[1], r[1], fma(r[0], r[0], eps2)));
            if (SKIPSELF && (jt + q) == k) r2 = 1.0;  // r, v, a, jr and gh are all zero here
            double *xb = acc, *vb = acc + 3;
            double *ab = ORDER >= 2 ? acc + 6 : acc;    // unused for order 1
            double *jb = ORDER == 3 ? acc + 9 : acc;    // unused below order 3
            pair_vjp<ORDER>(r, v, a, jr, r2, gh, gj, xb, vb, ab, jb, acc[NOUT - 1]);
        }
#pragma unroll
        for (int q = 0; q < NOUT; ++q) {
            two_sum_into(hi[q], lo[q], acc[q]);
            acc[q] = 0.0;
        }
    }
    if (k < n) {
        const int64_t soff = (int64_t)blockIdx.y * slice_stride;
#pragma unroll
        for (int q = 0; q < NOUT; ++q) {
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

template <int ORDER>
hipError_t launch_vjp_order(h6_ctx ctx, const SrcPtrs &src, const CotPtrs &cot, int n,
                            const OutPtrs &out, unsigned acc_mask) {
    constexpr int BLOCK = 128;
    constexpr int NOUT = VTraits<ORDER>::NOUT;
    const int blocks_i = ceil_div_i(n, BLOCK);
    int split = balanced_split(ctx, 2, BLOCK, n, blocks_i);
    const int64_t cap = ctx->partial_cap / ((int64_t)NOUT * n);
    if (split > cap) split = (int)std::max<int64_t>(1, cap);
    int slice_len = ceil_div_i(ceil_div_i(n, split), BLOCK) * BLOCK;
    split = ceil_div_i(n, slice_len);
    OutPtrs dst;
    int64_t slice_stride = 0;
    unsigned mask = acc_mask;
    if (split == 1) {
        dst = out;
    } else {
        for (int c = 0; c < kMaxOut; ++c) dst.p[c] = nullptr;
        for (int c = 0; c < NOUT; ++c) dst.p[c] = ctx->partial + (int64_t)c * n;
        slice_stride = (int64_t)NOUT * n;
        mask = 0u;  // partials are overwritten; the reduction applies acc_mask
    }
    dim3 grid(blocks_i, split);
    if (ctx->eps2 == 0.0)
        hipLaunchKernelGGL((k_eval_vjp<ORDER, BLOCK, true>), grid, dim3(BLOCK), 0, ctx->stream, src,
                           cot, n, ctx->eps2, slice_len, dst, slice_stride, mask);
    else
        hipLaunchKernelGGL((k_eval_vjp<ORDER, BLOCK, false>), grid, dim3(BLOCK), 0, ctx->stream,
                           src, cot, n, ctx->eps2, slice_len, dst, slice_stride, mask);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || split == 1) return e;
    return launch_reduce(ctx, split, NOUT, 0, n, out, acc_mask);
}

}  // namespace

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

}  // namespace h6
