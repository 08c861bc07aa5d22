// Integrator steps around the evaluation: predictor, corrector with
// interpolation and time-step assignment, start-up steps, the block
// scheduler, and the energy / angular momentum diagnostic.
//
// All of these are bandwidth- or latency-bound elementwise passes over
// structure-of-arrays FP64 data: one particle per lane, coalesced loads
// and stores, no LDS except for block-level reductions.
#include <algorithm>

#include "steps_body.h"

namespace h6 {
namespace {

using namespace stepbody;

__global__ __launch_bounds__(256) void k_predict(h6_state st, int n, int64_t t_tick, double dt,
                                                 int shared, h6_pred out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double d = shared ? dt : (double)(t_tick - st.t[i]) * kTick;
    predict_one(st, i, d, out);
}

template <bool SHARED>
__global__ __launch_bounds__(256) void k_correct(h6_state st, const int32_t *__restrict__ active,
                                                 int n_act, h6_force f, int64_t t_next, double dt_sh,
                                                 double eta6, int lev_min, int lev_max,
                                                 int32_t *flags) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_act) return;
    const int i = SHARED ? k : active[k];
    double fa[3], fj[3], fs[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        fa[c] = f.a[c][k];
        fj[c] = f.j[c][k];
        fs[c] = f.s[c][k];
    }
    correct_one<SHARED>(st, i, fa, fj, fs, t_next, dt_sh, eta6, lev_min, lev_max, flags);
}

// ---------------------------------------------------------------- start-up steps
// dt^2 = eta_s^2 (|a||s| + |j|^2) / (|j||c| + |s|^2)  (4th-order criterion)
__global__ __launch_bounds__(256) void k_initial_steps(h6_state st, int n, double eta2, int lev_min,
                                                       int lev_max, int32_t *flags) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a0 = st.a[0][i], a1 = st.a[1][i], a2 = st.a[2][i];
    const double j0 = st.j[0][i], j1 = st.j[1][i], j2 = st.j[2][i];
    const double s0 = st.s[0][i], s1 = st.s[1][i], s2 = st.s[2][i];
    const double c0 = st.c[0][i], c1 = st.c[1][i], c2 = st.c[2][i];
    const double num = fma(norm3(a0, a1, a2), norm3(s0, s1, s2), fma(j0, j0, fma(j1, j1, j2 * j2)));
    const double den = fma(norm3(j0, j1, j2), norm3(c0, c1, c2), fma(s0, s0, fma(s1, s1, s2 * s2)));
    int L = level_from_power((num / den) * eta2, 2, lev_min, lev_max + 1);
    if (L > lev_max) {
        atomicOr(flags, kFlagDtMin);
        L = lev_max;
    }
    st.t[i] = 0;
    st.dt[i] = (int64_t)1 << (kTickBits - L);
}

// ---------------------------------------------------------------- scheduler
// Two passes over fixed chunks of kSchedChunk particles per workgroup:
//   1. each chunk finds its minimum due time t + dt and how many of its
//      particles are due then; the last workgroup to finish takes the
//      global minimum t_next, gives every chunk whose minimum equals t_next
//      an offset (exclusive scan of their counts, in chunk order) and
//      publishes t_next and n_act;
//   2. each such chunk writes its due particles, in index order, at its
//      offset.
constexpr int kSchedThreads = 256;
constexpr int kSchedChunk = kSchedThreads * 16;

// Ordered hand-off between workgroups of one launch: every workgroup
// publishes its result, then increments the counter with a device-scope
// release; the one that sees count == nblocks - 1 is the last, acquires,
// and may read all published results. It resets the counter for the next
// launch.
__device__ __forceinline__ bool last_workgroup(unsigned *counter, unsigned nblocks) {
    __shared__ bool is_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev =
            __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        is_last = (prev == nblocks - 1);
        if (is_last) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last;
}

template <typename T>
__device__ __forceinline__ T load_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int64_t wave_min_i64(int64_t v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int64_t o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ int64_t block_min_i64(int64_t v) {
    __shared__ int64_t wmin[kSchedThreads / 64];
    v = wave_min_i64(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) wmin[w] = v;
    __syncthreads();
    int64_t r = wmin[0];
#pragma unroll
    for (int q = 1; q < kSchedThreads / 64; ++q) r = wmin[q] < r ? wmin[q] : r;
    __syncthreads();
    return r;
}

__device__ __forceinline__ int block_sum_i32(int v) {
    __shared__ int wsum[kSchedThreads / 64];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = 0;
#pragma unroll
    for (int q = 0; q < kSchedThreads / 64; ++q) r += wsum[q];
    __syncthreads();
    return r;
}

// out[0] = t_next, out[1] = n_act (the 16 bytes the host reads back)
__global__ __launch_bounds__(kSchedThreads) void k_sched_select(const int64_t *__restrict__ t,
                                                                const int64_t *__restrict__ dt,
                                                                int n, int64_t *chunk_min,
                                                                int32_t *chunk_cnt,
                                                                int32_t *chunk_off,
                                                                unsigned *counter, int64_t *out) {
    const int base = blockIdx.x * kSchedChunk;
    const int end = min(n, base + kSchedChunk);
    int64_t v = INT64_MAX;
    for (int i = base + threadIdx.x; i < end; i += kSchedThreads) {
        const int64_t due = t[i] + dt[i];
        v = due < v ? due : v;
    }
    const int64_t cmin = block_min_i64(v);
    int cnt = 0;
    for (int i = base + threadIdx.x; i < end; i += kSchedThreads) cnt += (t[i] + dt[i] == cmin);
    cnt = block_sum_i32(cnt);
    if (threadIdx.x == 0) {
        chunk_min[blockIdx.x] = cmin;
        chunk_cnt[blockIdx.x] = cnt;
    }
    if (!last_workgroup(counter, gridDim.x)) return;
    int64_t r = INT64_MAX;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += kSchedThreads) {
        const int64_t x = load_agent(&chunk_min[b]);
        r = x < r ? x : r;
    }
    r = block_min_i64(r);
    if (threadIdx.x == 0) {
        // exclusive scan over the (few hundred at most) chunks that hold t_next
        int run = 0;
        for (int b = 0; b < (int)gridDim.x; ++b) {
            const bool has = load_agent(&chunk_min[b]) == r;
            chunk_off[b] = has ? run : -1;
            run += has ? load_agent(&chunk_cnt[b]) : 0;
        }
        out[0] = r;
        out[1] = run;
    }
}

__global__ __launch_bounds__(kSchedThreads) void k_sched_compact(const int64_t *__restrict__ t,
                                                                 const int64_t *__restrict__ dt,
                                                                 int n, const int64_t *sel,
                                                                 const int32_t *chunk_off,
                                                                 int32_t *active) {
    __shared__ int wcnt[kSchedThreads / 64];
    const int off0 = chunk_off[blockIdx.x];
    if (off0 < 0) return;  // no particle of this chunk is due
    const int64_t tn = sel[0];
    const int base = blockIdx.x * kSchedChunk;
    const int end = min(n, base + kSchedChunk);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int run = off0;
    for (int r = base; r < end; r += kSchedThreads) {
        const int i = r + threadIdx.x;
        const bool due = i < end && (t[i] + dt[i] == tn);
        const unsigned long long mask = __ballot(due);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wcnt[w] = __popcll(mask);
        __syncthreads();
        int woff = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < kSchedThreads / 64; ++q) {
            woff += q < w ? wcnt[q] : 0;
            tot += wcnt[q];
        }
        if (due) active[run + woff + before] = i;
        run += tot;
        __syncthreads();
    }
}

// ---------------------------------------------------------------- energy
constexpr int kEnergyThreads = 256;
constexpr int kEnergyMaxSplit = 16;  // source slices per target block

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    const double bp = s - a;
    e = (a - (s - bp)) + (b - bp);
}

// Potential energy W = -sum over pairs i < j of m_i m_j / sqrt(r^2+eps^2),
// each pair once: target block b (kEnergyThreads particles, one per thread)
// meets the source tiles t >= b, and in its own tile only the sources
// j > i. Blocks b and nb-1-b share a workgroup, so that every workgroup has
// nb + 1 tiles of work (the middle block of an odd nb alone has fewer); the
// tiles are cut into gridDim.y slices. Sums over a tile are plain, over
// tiles compensated. Kinetic m v^2/2 and angular momentum m x cross v of
// the workgroup's particles are taken by the first slice. Workgroup sums as
// compensated (hi, lo) trees; the last workgroup adds them in order.
__global__ __launch_bounds__(kEnergyThreads) void k_energy(h6_state st, int n, double eps2,
                                                           double *partial, unsigned *counter,
                                                           double *out) {
    __shared__ double4 tile[kEnergyThreads];  // x, y, z, m
    __shared__ double red_hi[5][kEnergyThreads];
    __shared__ double red_lo[5][kEnergyThreads];
    const int tid = threadIdx.x;
    const int nb = (n + kEnergyThreads - 1) / kEnergyThreads;
    const int b0 = (int)blockIdx.x, b1 = nb - 1 - (int)blockIdx.x;
    const bool two = b1 > b0;
    const int nt0 = nb - b0, nt = nt0 + (two ? nb - b1 : 0);
    const int vt0 = (int)(((int64_t)blockIdx.y * nt) / gridDim.y);
    const int vt1 = (int)(((int64_t)(blockIdx.y + 1) * nt) / gridDim.y);
    const int i0 = b0 * kEnergyThreads + tid, i1 = b1 * kEnergyThreads + tid;
    const int c0 = i0 < n ? i0 : n - 1, c1 = i1 < n ? i1 : n - 1;
    const double p0x = st.x[0][c0], p0y = st.x[1][c0], p0z = st.x[2][c0];
    const double p1x = st.x[0][c1], p1y = st.x[1][c1], p1z = st.x[2][c1];
    double phi0_hi = 0.0, phi0_lo = 0.0, phi1_hi = 0.0, phi1_lo = 0.0;
    for (int vt = vt0; vt < vt1; ++vt) {
        const bool first = vt < nt0;  // a tile of block b0 (else of b1)
        const int b = first ? b0 : b1;
        const int t = first ? b0 + vt : b1 + (vt - nt0);
        __syncthreads();
        const int jj = t * kEnergyThreads + tid;
        tile[tid] = jj < n ? make_double4(st.x[0][jj], st.x[1][jj], st.x[2][jj], st.m[jj])
                           : make_double4(1.0e18, 1.0e18, 1.0e18, 0.0);
        __syncthreads();
        const double xi0 = first ? p0x : p1x, xi1 = first ? p0y : p1y, xi2 = first ? p0z : p1z;
        double acc = 0.0;
        if (t == b) {  // own tile: sources after the target only
#pragma unroll 4
            for (int q = 0; q < kEnergyThreads; ++q) {
                const double4 r = tile[q];
                const double dx = r.x - xi0, dy = r.y - xi1, dz = r.z - xi2;
                double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
                const bool take = q > tid;
                r2 = take ? r2 : 1.0;
                acc = fma(take ? r.w : 0.0, rsqrt_f64(r2), acc);
            }
        } else {
#pragma unroll 4
            for (int q = 0; q < kEnergyThreads; ++q) {
                const double4 r = tile[q];
                const double dx = r.x - xi0, dy = r.y - xi1, dz = r.z - xi2;
                const double r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
                acc = fma(r.w, rsqrt_f64(r2), acc);
            }
        }
        double s, e;
        if (first) {
            two_sum(phi0_hi, acc, s, e);
            phi0_hi = s;
            phi0_lo += e;
        } else {
            two_sum(phi1_hi, acc, s, e);
            phi1_hi = s;
            phi1_lo += e;
        }
    }
    double v[5] = {0, 0, 0, 0, 0};
    const bool has0 = i0 < n, has1 = two && i1 < n;
    if (has0) v[1] = -st.m[i0] * (phi0_hi + phi0_lo);
    if (has1) v[1] = fma(-st.m[i1], phi1_hi + phi1_lo, v[1]);
    if (blockIdx.y == 0) {
        if (has0) {
            const double m = st.m[i0], vx = st.v[0][i0], vy = st.v[1][i0], vz = st.v[2][i0];
            v[0] = 0.5 * m * fma(vx, vx, fma(vy, vy, vz * vz));
            v[2] = m * (p0y * vz - p0z * vy);
            v[3] = m * (p0z * vx - p0x * vz);
            v[4] = m * (p0x * vy - p0y * vx);
        }
        if (has1) {
            const double m = st.m[i1], vx = st.v[0][i1], vy = st.v[1][i1], vz = st.v[2][i1];
            v[0] += 0.5 * m * fma(vx, vx, fma(vy, vy, vz * vz));
            v[2] += m * (p1y * vz - p1z * vy);
            v[3] += m * (p1z * vx - p1x * vz);
            v[4] += m * (p1x * vy - p1y * vx);
        }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        red_hi[q][tid] = v[q];
        red_lo[q][tid] = 0.0;
    }
    __syncthreads();
    for (int w = kEnergyThreads / 2; w >= 1; w >>= 1) {
        if (tid < w) {
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                double s, e;
                two_sum(red_hi[q][tid], red_hi[q][tid + w], s, e);
                red_hi[q][tid] = s;
                red_lo[q][tid] += red_lo[q][tid + w] + e;
            }
        }
        __syncthreads();
    }
    const int wg = (int)(blockIdx.y * gridDim.x + blockIdx.x);
    const int n_wg = (int)(gridDim.x * gridDim.y);
    if (tid < 5) {
        partial[2 * (wg * 5 + tid)] = red_hi[tid][0];
        partial[2 * (wg * 5 + tid) + 1] = red_lo[tid][0];
    }
    if (!last_workgroup(counter, n_wg)) return;
    // the last workgroup: every thread takes every 256th workgroup sum, then
    // the same fixed tree (deterministic for a launch shape)
    double hi[5] = {0, 0, 0, 0, 0}, lo[5] = {0, 0, 0, 0, 0};
    for (int b = tid; b < n_wg; b += kEnergyThreads) {
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            double s, e;
            two_sum(hi[q], load_agent(&partial[2 * (b * 5 + q)]), s, e);
            hi[q] = s;
            lo[q] += e + load_agent(&partial[2 * (b * 5 + q) + 1]);
        }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        red_hi[q][tid] = hi[q];
        red_lo[q][tid] = lo[q];
    }
    __syncthreads();
    for (int w = kEnergyThreads / 2; w >= 1; w >>= 1) {
        if (tid < w) {
#pragma unroll
            for (int q = 0; q < 5; ++q) {
                double s, e;
                two_sum(red_hi[q][tid], red_hi[q][tid + w], s, e);
                red_hi[q][tid] = s;
                red_lo[q][tid] += red_lo[q][tid + w] + e;
            }
        }
        __syncthreads();
    }
    if (tid < 5) out[tid] = red_hi[tid][0] + red_lo[tid][0];
}

}  // namespace

int sched_blocks_for(int64_t n) { return (int)((n + kSchedChunk - 1) / kSchedChunk); }
// workgroup partial slots for n particles (target blocks x the most slices)
int energy_blocks_for(int64_t n) {
    return (int)((n + kEnergyThreads - 1) / kEnergyThreads) * kEnergyMaxSplit;
}

hipError_t launch_predict(h6_ctx ctx, const h6_state *st, int n, int64_t t_tick, double dt,
                          bool shared, const h6_pred *out) {
    hipLaunchKernelGGL(k_predict, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, *st, n, t_tick,
                       dt, shared ? 1 : 0, *out);
    return hipGetLastError();
}

hipError_t launch_correct(h6_ctx ctx, h6_state *st, const int32_t *active, int n_act,
                          const h6_force *f, int64_t t_next, double dt, const h6_params *prm,
                          bool shared) {
    if (n_act <= 0) return hipSuccess;
    dim3 grid((n_act + 255) / 256);
    if (shared) {
        hipLaunchKernelGGL(k_correct<true>, grid, dim3(256), 0, ctx->stream, *st, active, n_act, *f,
                           (int64_t)0, dt, 0.0, 0, 0, ctx->flags);
    } else {
        const double e = prm->eta, e2 = e * e;
        hipLaunchKernelGGL(k_correct<false>, grid, dim3(256), 0, ctx->stream, *st, active, n_act,
                           *f, t_next, 0.0, e2 * e2 * e2, prm->lev_min, prm->lev_max, ctx->flags);
    }
    return hipGetLastError();
}

hipError_t launch_initial_steps(h6_ctx ctx, h6_state *st, int n, double eta_s, int lev_min,
                                int lev_max) {
    hipLaunchKernelGGL(k_initial_steps, dim3((n + 255) / 256), dim3(256), 0, ctx->stream, *st, n,
                       eta_s * eta_s, lev_min, lev_max, ctx->flags);
    return hipGetLastError();
}

// Scratch layout: ctx->sched64[0..1] = {t_next, n_act} (read back by the
// host), ctx->sched64[2..] chunk minima; ctx->sched32[0..nb) chunk counts,
// [nb..2nb) chunk offsets; counters[0] is the hand-off counter.
hipError_t launch_next_block(h6_ctx ctx, const h6_state *st, int n, int32_t *active) {
    const int nb = sched_blocks_for(n);
    int64_t *sel = ctx->sched64;
    int64_t *cmin = ctx->sched64 + 2;
    int32_t *ccnt = ctx->sched32;
    int32_t *coff = ctx->sched32 + nb;
    hipLaunchKernelGGL(k_sched_select, dim3(nb), dim3(kSchedThreads), 0, ctx->stream, st->t, st->dt,
                       n, cmin, ccnt, coff, ctx->counters, sel);
    hipLaunchKernelGGL(k_sched_compact, dim3(nb), dim3(kSchedThreads), 0, ctx->stream, st->t,
                       st->dt, n, (const int64_t *)sel, (const int32_t *)coff, active);
    return hipGetLastError();
}

hipError_t launch_energy(h6_ctx ctx, const h6_state *st, int n) {
    const int nb = (n + kEnergyThreads - 1) / kEnergyThreads;
    const int pairs = (nb + 1) / 2;  // workgroups per slice: blocks b and nb-1-b together
    // about four workgroups of four waves per compute unit, at most one
    // slice per tile of a workgroup's nb + 1
    int split = std::max(1, std::min(kEnergyMaxSplit, (4 * ctx->n_cu + pairs - 1) / pairs));
    split = std::min(split, nb + 1);
    hipLaunchKernelGGL(k_energy, dim3(pairs, split), dim3(kEnergyThreads), 0, ctx->stream, *st, n,
                       ctx->eps2, ctx->ered + 8, ctx->counters + 2, ctx->ered);
    return hipGetLastError();
}

}  // namespace h6
