// Device-resident block stepping: the kernels of one block step read the
// block time and active count from device memory, so the host enqueues
// blocks back to back and synchronises once per batch of blocks instead of
// once per block (the paper's code synchronises host and device every
// step, Sec. 3 item 3; at block-step granularity that round trip would
// cost more than the small blocks' arithmetic).
//
// Per block, in stream order:
//   k_bl_select     chunk minima and tie counts of t + dt; the last
//                   workgroup publishes t_next, n_act and the evaluation's
//                   launch shape in a BlockDesc (n_act = 0 once t_next would
//                   pass t_end: the block and all later ones become no-ops)
//   k_bl_compact_predict  every particle predicted to t_next, and the
//                   active list in index order
//   k_bl_eval       fixed grid; each workgroup takes its (target group,
//                   source slice) units from the BlockDesc
//   k_bl_reduce_correct  compensated slice sums, then the corrector and
//                   step rule for each active particle
// The arithmetic is that of the host-sequenced path (shared bodies).
#include "eval_body.h"
#include "eval_mixed_body.h"
#include "steps_body.h"

namespace h6 {
namespace {

using namespace evalbody;
using namespace mixedbody;
using namespace stepbody;

constexpr int kSelThreads = 256;
constexpr int kSelChunk = 1024;  // particles per workgroup in select/compact
constexpr int kSmall1Max = 16;   // active sets up to this size: one target per wave
constexpr int kSmall2Max = 128;  // up to this size: source-parallel, two targets per wave
constexpr int kTileBlock = 64;   // tile kernel: one wave, two targets per lane
constexpr int kTileIpl = 2;
constexpr int kWaveReduce = 24;  // slices from which one wave reduces one target

__device__ __forceinline__ int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Exclusive prefix sum over the 256 threads of a workgroup; *total gets
// the sum. Wave scans by shuffles, then the four wave totals.
__device__ __forceinline__ int block_excl_scan(int v, int *total) {
    __shared__ int wsum[kSelThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int inc = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_up(inc, off, 64);
        if (lane >= off) inc += o;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int q = 0; q < kSelThreads / 64; ++q) {
        before += q < w ? wsum[q] : 0;
        all += wsum[q];
    }
    __syncthreads();
    *total = all;
    return before + inc - v;
}

__device__ __forceinline__ int64_t block_min(int64_t v) {
    __shared__ int64_t wmin[kSelThreads / 64];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int64_t o = __shfl_xor(v, off, 64);
        v = o < v ? o : v;
    }
    if ((threadIdx.x & 63) == 0) wmin[threadIdx.x >> 6] = v;
    __syncthreads();
    int64_t r = wmin[0];
#pragma unroll
    for (int q = 1; q < kSelThreads / 64; ++q) r = wmin[q] < r ? wmin[q] : r;
    __syncthreads();
    return r;
}

__device__ __forceinline__ int block_sum(int v) {
    int total;
    (void)block_excl_scan(v, &total);
    return total;
}

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

// Launch shape of the evaluation for n_act targets (written into the
// BlockDesc). Source-parallel kinds (1: one target per wave, 3: two): slices
// of at least 256 sources (4 per lane), at most eval_grid waves in all.
// Tile kind 0 (128 targets per one-wave workgroup): the largest slice
// count whose units fit one round of resident workgroups (eval_grid), at
// least four 64-source tiles per slice. Bounded by the partial capacity.
__device__ void launch_shape(BlockDesc &d, int n, int n_act, int eval_grid, int64_t partial_cap) {
    int split;
    if (n_act <= kSmall2Max) {
        d.kind = n_act <= kSmall1Max ? 1 : 3;
        d.groups = d.kind == 1 ? n_act : cdiv(n_act, 2);
        split = cdiv(n, 256);
        const int fit = eval_grid / d.groups;
        split = split < fit ? split : fit;
    } else {
        d.kind = 0;
        d.groups = cdiv(n_act, kTileBlock * kTileIpl);
        split = eval_grid / d.groups;
        const int cap = n / (4 * kTileBlock);
        split = split < cap ? split : cap;
    }
    const int64_t pc = partial_cap / ((int64_t)9 * n_act);
    if (split > pc) split = (int)pc;
    if (split < 1) split = 1;
    int slice = cdiv(cdiv(n, split), 64) * 64;
    d.slice_len = slice;
    d.split = cdiv(n, slice);
}

__global__ __launch_bounds__(kSelThreads) void k_bl_select(
    const int64_t *__restrict__ t, const int64_t *__restrict__ dt, int n, int64_t t_end,
    int64_t *chunk_min, int32_t *chunk_cnt, int32_t *chunk_off, unsigned *counter, BlockDesc *desc,
    int32_t *nact_log, int log_mask, int64_t seq, int eval_grid, int64_t partial_cap) {
    const int base = blockIdx.x * kSelChunk;
    const int end = min(n, base + kSelChunk);
    int64_t v = INT64_MAX;
    for (int i = base + threadIdx.x; i < end; i += kSelThreads) {
        const int64_t due = t[i] + dt[i];
        v = due < v ? due : v;
    }
    const int64_t cmin = block_min(v);
    int cnt = 0;
    for (int i = base + threadIdx.x; i < end; i += kSelThreads) cnt += (t[i] + dt[i] == cmin);
    cnt = block_sum(cnt);
    if (threadIdx.x == 0) {
        chunk_min[blockIdx.x] = cmin;
        chunk_cnt[blockIdx.x] = cnt;
    }
    if (!last_workgroup(counter, gridDim.x)) return;
    const int nb = gridDim.x;
    int64_t r = INT64_MAX;
    for (int b = threadIdx.x; b < nb; b += kSelThreads) {
        const int64_t x = load_agent(&chunk_min[b]);
        r = x < r ? x : r;
    }
    r = block_min(r);
    // offsets of the chunks holding t_next: each thread scans a run of chunks
    const int per = cdiv(nb, kSelThreads);
    const int b0 = threadIdx.x * per;
    int mine = 0;
    for (int b = b0; b < b0 + per && b < nb; ++b)
        mine += load_agent(&chunk_min[b]) == r ? load_agent(&chunk_cnt[b]) : 0;
    int total;
    int run = block_excl_scan(mine, &total);
    for (int b = b0; b < b0 + per && b < nb; ++b) {
        const bool has = load_agent(&chunk_min[b]) == r;
        chunk_off[b] = has ? run : -1;
        run += has ? load_agent(&chunk_cnt[b]) : 0;
    }
    if (threadIdx.x == 0) {
        BlockDesc d = *desc;
        const bool past = r > t_end;
        d.t_next = r;
        d.n_act = past ? 0 : total;
        d.done = past ? 1 : 0;
        if (!past) {
            launch_shape(d, n, total, eval_grid, partial_cap);
            d.blocks += 1;
            d.particle_steps += total;
        }
        if (nact_log) nact_log[seq & log_mask] = d.n_act;
        *desc = d;
    }
}

// Predicts every particle of the chunk to t_next, and writes the chunk's
// due particles, in index order, at the chunk's offset in the active list.
__global__ __launch_bounds__(kSelThreads) void k_bl_compact_predict(h6_state st, int n,
                                                                    const BlockDesc *desc,
                                                                    const int32_t *chunk_off,
                                                                    int32_t *active, h6_pred out) {
    __shared__ int wcnt[kSelThreads / 64];
    if (desc->n_act == 0) return;
    const int64_t tn = desc->t_next;
    const int base = blockIdx.x * kSelChunk;
    const int end = min(n, base + kSelChunk);
    for (int i = base + threadIdx.x; i < end; i += kSelThreads)
        predict_one(st, i, (double)(tn - st.t[i]) * kTick, out);
    const int off0 = chunk_off[blockIdx.x];
    if (off0 < 0) return;  // no particle of this chunk is due
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int run = off0;
    for (int r = base; r < end; r += kSelThreads) {
        const int i = r + threadIdx.x;
        const bool due = i < end && (st.t[i] + st.dt[i] == tn);
        const unsigned long long mask = __ballot(due);
        const int before = __popcll(mask & ((1ull << lane) - 1ull));
        if (lane == 0) wcnt[w] = __popcll(mask);
        __syncthreads();
        int woff = 0, tot = 0;
#pragma unroll
        for (int q = 0; q < kSelThreads / 64; ++q) {
            woff += q < w ? wcnt[q] : 0;
            tot += wcnt[q];
        }
        if (due) active[run + woff + before] = i;
        run += tot;
        __syncthreads();
    }
}

template <bool MIXED, bool SKIPSELF>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_bl_eval(
    SrcPtrs src, const int32_t *__restrict__ active, int n, double eps2, const BlockDesc *desc,
    double *partial, OutPtrs force) {
    const int n_act = desc->n_act;
    if (n_act == 0) return;
    const int split = desc->split, slice_len = desc->slice_len, groups = desc->groups;
    const int kind = desc->kind;
    OutPtrs out;
    int64_t slice_stride = 0;
    if (split == 1) {
        out = force;
    } else {
#pragma unroll
        for (int c = 0; c < kMaxOut; ++c) out.p[c] = c < 9 ? partial + (int64_t)c * n_act : nullptr;
        slice_stride = (int64_t)9 * n_act;
    }
    const int units = groups * split;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int g = u / split, sl = u - g * split;
        if (kind == 1) {
            if constexpr (MIXED)
                mixed_small_body<1, SKIPSELF>(src, active, n, n_act, eps2, slice_len, out,
                                              slice_stride, g, sl);
            else
                eval_small_body<1, SKIPSELF>(src, active, n, n_act, eps2, slice_len, out,
                                             slice_stride, g, sl);
        } else if (kind == 3) {
            if constexpr (MIXED)
                mixed_small_body<2, SKIPSELF>(src, active, n, n_act, eps2, slice_len, out,
                                              slice_stride, g, sl);
            else
                eval_small_body<2, SKIPSELF>(src, active, n, n_act, eps2, slice_len, out,
                                             slice_stride, g, sl);
        } else {
            if constexpr (MIXED)
                mixed_tile_body<kTileBlock, kTileIpl, SKIPSELF>(src, active, n, n_act, eps2,
                                                                slice_len, out, slice_stride, g, sl);
            else
                eval_tile_body<2, kTileBlock, kTileIpl, SKIPSELF>(src, active, n, n_act, eps2,
                                                                  slice_len, out, slice_stride, g,
                                                                  sl);
        }
    }
}

__device__ __forceinline__ void neumaier(double &s, double &c, double x) {
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
}

// Slice sums (if any) and the corrector for every active particle. Few
// slices: one thread per target, sums in slice order; many slices: one
// wave per target, lanes over slices, fixed butterfly. The reduced forces
// are also stored in `force` (active order).
__global__ __launch_bounds__(256) void k_bl_reduce_correct(h6_state st,
                                                           const int32_t *__restrict__ active,
                                                           const BlockDesc *desc,
                                                           const double *__restrict__ partial,
                                                           OutPtrs force, double eta6, int lev_min,
                                                           int lev_max, int32_t *flags) {
    const int n_act = desc->n_act;
    if (n_act == 0) return;
    const int split = desc->split;
    const int64_t tn = desc->t_next;
    if (split < kWaveReduce) {
        for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n_act;
             k += gridDim.x * blockDim.x) {
            double f[9];
            if (split == 1) {
#pragma unroll
                for (int c = 0; c < 9; ++c) f[c] = force.p[c][k];
            } else {
#pragma unroll
                for (int c = 0; c < 9; ++c) {
                    double s = 0.0, comp = 0.0;
                    for (int sl = 0; sl < split; ++sl)
                        neumaier(s, comp, partial[((int64_t)sl * 9 + c) * n_act + k]);
                    f[c] = s + comp;
                    force.p[c][k] = f[c];
                }
            }
            correct_one<false>(st, active[k], f, f + 3, f + 6, tn, 0.0, eta6, lev_min, lev_max,
                               flags);
        }
        return;
    }
    const int lane = threadIdx.x & 63;
    const int waves = gridDim.x * (blockDim.x >> 6);
    for (int k = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); k < n_act; k += waves) {
        double f[9];
#pragma unroll
        for (int c = 0; c < 9; ++c) {
            double s = 0.0, comp = 0.0;
            for (int sl = lane; sl < split; sl += 64)
                neumaier(s, comp, partial[((int64_t)sl * 9 + c) * n_act + k]);
            wave_comp_sum(s, comp);
            f[c] = s + comp;
        }
        if (lane == 0) {
#pragma unroll
            for (int c = 0; c < 9; ++c) force.p[c][k] = f[c];
            correct_one<false>(st, active[k], f, f + 3, f + 6, tn, 0.0, eta6, lev_min, lev_max,
                               flags);
        }
    }
}

__global__ void k_bl_reset(BlockDesc *desc) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        BlockDesc d = {};
        *desc = d;
    }
}

}  // namespace

int bl_select_blocks(int64_t n) { return (int)((n + kSelChunk - 1) / kSelChunk); }
int bl_eval_grid(h6_ctx ctx) { return ctx->n_cu * 8; }  // one round of resident tile workgroups

hipError_t bl_reset(h6_ctx ctx) {
    hipLaunchKernelGGL(k_bl_reset, dim3(1), dim3(64), 0, ctx->stream, ctx->bl_desc);
    return hipGetLastError();
}

hipError_t bl_enqueue_block(h6_ctx ctx, h6_state *st, int n, const h6_pred *pred,
                            const h6_force *f, int32_t *active, const h6_params *prm,
                            int64_t t_end, int64_t seq) {
    const int nb = bl_select_blocks(n);
    int64_t *cmin = ctx->sched64 + 2;
    int32_t *ccnt = ctx->sched32;
    int32_t *coff = ctx->sched32 + nb;
    const int eval_grid = bl_eval_grid(ctx);
    hipLaunchKernelGGL(k_bl_select, dim3(nb), dim3(kSelThreads), 0, ctx->stream, st->t, st->dt, n,
                       t_end, cmin, ccnt, coff, ctx->counters + 3, ctx->bl_desc, ctx->bl_log,
                       ctx->bl_log_mask, seq, eval_grid, ctx->partial_cap);
    hipLaunchKernelGGL(k_bl_compact_predict, dim3(nb), dim3(kSelThreads), 0, ctx->stream, *st, n,
                       (const BlockDesc *)ctx->bl_desc, (const int32_t *)coff, active, *pred);
    SrcPtrs src;
    for (int c = 0; c < 3; ++c) {
        src.x[c] = pred->x[c];
        src.v[c] = pred->v[c];
        src.a[c] = pred->a[c];
        src.j[c] = nullptr;
    }
    src.m = st->m;
    OutPtrs fo;
    for (int c = 0; c < kMaxOut; ++c) fo.p[c] = nullptr;
    for (int c = 0; c < 3; ++c) {
        fo.p[c] = f->a[c];
        fo.p[3 + c] = f->j[c];
        fo.p[6 + c] = f->s[c];
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (ctx->prof) {
        hipError_t pe = prof_begin(ctx, &ev0, &ev1);
        if (pe != hipSuccess) return pe;
    }
    const bool skip = ctx->eps2 == 0.0;
    const bool mixed = prm->precision == H6_MIXED;
#define H6_BL_EVAL(M, S)                                                                          \
    hipLaunchKernelGGL((k_bl_eval<M, S>), dim3(eval_grid), dim3(64), 0, ctx->stream, src, active, \
                       n, ctx->eps2, (const BlockDesc *)ctx->bl_desc, ctx->partial, fo)
    if (mixed) {
        if (skip) H6_BL_EVAL(true, true); else H6_BL_EVAL(true, false);
    } else {
        if (skip) H6_BL_EVAL(false, true); else H6_BL_EVAL(false, false);
    }
#undef H6_BL_EVAL
    if (ctx->prof) {
        hipError_t pe = hipGetLastError();
        if (pe != hipSuccess) return pe;
        pe = prof_end_seq(ctx, ev0, ev1, prm->precision, seq);
        if (pe != hipSuccess) return pe;
    }
    const double e = prm->eta, e2 = e * e;
    hipLaunchKernelGGL(k_bl_reduce_correct, dim3(ctx->n_cu * 4), dim3(256), 0, ctx->stream, *st,
                       (const int32_t *)active, (const BlockDesc *)ctx->bl_desc,
                       (const double *)ctx->partial, fo, e2 * e2 * e2, prm->lev_min, prm->lev_max,
                       ctx->flags);
    return hipGetLastError();
}

}  // namespace h6
