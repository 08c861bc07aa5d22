// Device arithmetic helpers shared by the libh6 kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace h6 {

// 1/sqrt(r2): the hardware estimate v_rsq_f64 (relative error below about
// 5e-8 on gfx950, measured) refined by one Newton step,
//   e = 1 - r2 y^2,  y <- y + (y e) / 2,
// which takes a relative error d to (3/2) d^2 (from below): at most about
// 4e-15, a smooth function of r2 alone, so the force stays central and
// the summed a, j, s keep errors near 1e-14. Four operations besides the
// estimate (the third-order step costs five).
__device__ __forceinline__ double rsqrt_f64(double r2) {
    const double y = __builtin_amdgcn_rsq(r2);
    const double t = r2 * y;
    const double e = fma(-t, y, 1.0);
    const double ye = y * e;
    return fma(ye, 0.5, y);
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

// A double moved across lanes by a DPP lane pattern (both 32-bit halves);
// lanes of rows outside ROWS get 0.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_f64(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}

// One butterfly stage for NV compensated pairs: every lane merges its value
// with its partner's (partner value from DPP pattern CTRL, or from the lane
// at XOR distance `off` when CTRL < 0), the lower group's value first.
template <int NV, int CTRL>
__device__ __forceinline__ void comp_stage(double *s, double *c, bool upper, int off) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double s2, c2;
        if constexpr (CTRL >= 0) {
            s2 = dpp_f64<CTRL>(s[q]);
            c2 = dpp_f64<CTRL>(c[q]);
        } else {
            s2 = __shfl_xor(s[q], off, 64);
            c2 = __shfl_xor(c[q], off, 64);
        }
        double a = upper ? s2 : s[q], ac = upper ? c2 : c[q];
        const double b = upper ? s[q] : s2, bc = upper ? c[q] : c2;
        comp_merge(a, ac, b, bc);
        s[q] = a;
        c[q] = ac;
    }
}

// The butterfly for NV compensated pairs at once (stage by stage, so the NV
// exchanges of a stage are independent), within aligned segments of seg
// lanes (seg a power of two up to 64, uniform across the wave): every lane
// gets its segment's totals, the same in every lane and on every run.
// Stages pair lane groups of 1, 2, 4, 8, 16, 32 lanes. The first four stay
// within 16-lane rows and use DPP moves: quad permutations for the first
// two, then the half-row and row mirrors, which pair the two halves of each
// group of 8 (then 16) lanes; after the earlier stages every lane of a half
// holds the same value, so a mirror partner is as good as the XOR one.
template <int NV>
__device__ __forceinline__ void seg_comp_sum_n(double *s, double *c, int seg) {
    const int lane = threadIdx.x & 63;
    if (seg >= 2) comp_stage<NV, 0xB1>(s, c, (lane & 1) != 0, 1);    // quad_perm [1,0,3,2]
    if (seg >= 4) comp_stage<NV, 0x4E>(s, c, (lane & 2) != 0, 2);    // quad_perm [2,3,0,1]
    if (seg >= 8) comp_stage<NV, 0x141>(s, c, (lane & 4) != 0, 4);   // row_half_mirror
    if (seg >= 16) comp_stage<NV, 0x140>(s, c, (lane & 8) != 0, 8);  // row_mirror
    if (seg >= 32) comp_stage<NV, -1>(s, c, (lane & 16) != 0, 16);
    if (seg >= 64) comp_stage<NV, -1>(s, c, (lane & 32) != 0, 32);
}

// One row-broadcast stage for NV compensated pairs: the lanes of the rows in
// ROWS merge the value of the last lane of an earlier row (DPP row_bcast:15
// takes lane 15 of the row before, row_bcast:31 lane 31) into their own,
// the earlier rows' value first; the other rows merge zero (no change).
template <int NV, int CTRL, int ROWS>
__device__ __forceinline__ void bcast_stage(double *s, double *c) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
        double a = dpp_f64<CTRL, ROWS>(s[q]), ac = dpp_f64<CTRL, ROWS>(c[q]);
        comp_merge(a, ac, s[q], c[q]);
        s[q] = a;
        c[q] = ac;
    }
}

// Sums of NV compensated pairs within aligned segments of seg lanes (seg a
// power of two up to 64, uniform across the wave), valid in the LAST lane of
// each segment (deterministic for a given seg). Within 16-lane rows the
// butterfly of seg_comp_sum_n; across rows, instead of the two exchanges
// through LDS, two DPP row broadcasts: row_bcast:15 adds row 0 into row 1
// and row 2 into row 3, then (seg 64) row_bcast:31 adds rows 0-1 into
// rows 2-3, so that lane 63 holds the wave's total.
template <int NV>
__device__ __forceinline__ void seg_comp_reduce_n(double *s, double *c, int seg) {
    seg_comp_sum_n<NV>(s, c, seg < 16 ? seg : 16);
    if (seg >= 32) bcast_stage<NV, 0x142, 0xA>(s, c);  // row_bcast:15 into rows 1, 3
    if (seg >= 64) bcast_stage<NV, 0x143, 0xC>(s, c);  // row_bcast:31 into rows 2, 3
}

// Minimum of a 32-bit unsigned over each 16-lane row, by four DPP stages
// (the two quad permutations, then the half-row and row mirrors, which pair
// the halves of each group of 8, then 16 lanes once every lane of a half
// holds its half's minimum); every lane of a row ends with the row's
// minimum. All lanes of the wave must be active.
__device__ __forceinline__ unsigned row_min_u32(unsigned v) {
    int o;
    o = __builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
    v = (unsigned)o < v ? (unsigned)o : v;
    o = __builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
    v = (unsigned)o < v ? (unsigned)o : v;
    o = __builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    v = (unsigned)o < v ? (unsigned)o : v;
    o = __builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false);  // row_mirror
    v = (unsigned)o < v ? (unsigned)o : v;
    return v;
}

// Totals over the 64 lanes of a one-wave workgroup of NV values per lane,
// through LDS instead of a butterfly of compensated merges (which costs NV
// merges per stage and lane). On entry lds[v * 64 + lane] holds lane's value
// v (a compensated pair already rounded to one double). Lane (v, g) -- G =
// 64 / NV lanes per value -- sums every G-th lane's value v in lane order
// into a compensated pair, and lane v merges the G pairs of value v in
// order. Lane v < NV returns the total of value v, the other lanes 0; the
// result does not depend on timing. lds: 64 * NV doubles of workgroup
// memory (NV from 2 to 64); every thread of the workgroup calls it (it
// contains barriers).
template <int NV>
__device__ __forceinline__ double wave_totals_lds(double *lds) {
    static_assert(NV >= 2 && NV <= 64, "2 to 64 values per lane");
    constexpr int G = 64 / NV;
    const int lane = threadIdx.x & 63;
    __syncthreads();
    const int v = lane / G, g = lane - v * G;
    double hs = 0.0, hc = 0.0;
    if (v < NV) {
#pragma unroll
        for (int i = 0; i < (64 + G - 1) / G; ++i)
            if (g + i * G < 64) two_sum_into(hs, hc, lds[v * 64 + g + i * G]);
    }
    __syncthreads();
    if (v < NV) {
        lds[2 * lane] = hs;
        lds[2 * lane + 1] = hc;
    }
    __syncthreads();
    double total = 0.0;
    if (lane < NV) {
        double ts = 0.0, tc = 0.0;
#pragma unroll
        for (int q = 0; q < G; ++q)
            comp_merge(ts, tc, lds[2 * (lane * G + q)], lds[2 * (lane * G + q) + 1]);
        total = ts + tc;
    }
    return total;
}

}  // namespace h6
