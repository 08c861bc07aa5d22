// Device arithmetic helpers shared by the libh6 kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace h6 {

// 1/sqrt(r2): the hardware estimate v_rsq_f64 (relative error about 5e-8 on
// gfx950) refined by one third-order Newton step,
//   e = 1 - r2 y^2,  y <- y (1 + e/2 + 3 e^2/8),
// which takes a relative error d to about (5/2)(2d)^3, below double rounding.
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

// Compensated sum of (s1, c1) and (s2, c2): TwoSum of the leading parts,
// compensations added.
__device__ __forceinline__ void comp_merge(double &s, double &c, double s2, double c2) {
    const double t = s + s2;
    const double bp = t - s;
    const double err = (s - (t - bp)) + (s2 - bp);
    s = t;
    c += err + c2;
}

// Sum of a compensated pair over the 64 lanes of a wave by a fixed
// butterfly (both partners merge lower-lane value first), so the result is
// the same on every run; every lane ends with the total.
__device__ __forceinline__ void wave_comp_sum(double &s, double &c) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double s2 = __shfl_xor(s, off, 64);
        const double c2 = __shfl_xor(c, off, 64);
        double a = (lane & off) ? s2 : s, ac = (lane & off) ? c2 : c;
        const double b = (lane & off) ? s : s2, bc = (lane & off) ? c : c2;
        comp_merge(a, ac, b, bc);
        s = a;
        c = ac;
    }
}

// The same butterfly within aligned segments of seg lanes (seg a power of
// two up to 64, uniform across the wave): every lane gets its segment's
// total.
__device__ __forceinline__ void seg_comp_sum(double &s, double &c, int seg) {
    const int lane = threadIdx.x & 63;
    for (int off = seg >> 1; off >= 1; off >>= 1) {
        const double s2 = __shfl_xor(s, off, 64);
        const double c2 = __shfl_xor(c, off, 64);
        double a = (lane & off) ? s2 : s, ac = (lane & off) ? c2 : c;
        const double b = (lane & off) ? s : s2, bc = (lane & off) ? c : c2;
        comp_merge(a, ac, b, bc);
        s = a;
        c = ac;
    }
}

}  // namespace h6
