// Device-resident block stepping (block time steps, Sec. 2.2; host-device
// synchronisation per step, Sec. 3 item 3).
//
// Particles are kept in per-level lists (level L: step 2^-L). With
// power-of-two steps, every particle's time is the largest multiple of its
// own step not after the current block time t, so
//   t_next = min over occupied levels L of the next multiple of 2^-L after t,
// and the particles due at t_next are exactly those on the levels whose step
// divides t_next. Choosing a block is O(levels) work and its active set is a
// concatenation of whole lists: no pass over all particles per block.
//
// Lists: two buffers per level, capacity n each. During a block the active
// levels' lists are read (targets) from one buffer while the corrected
// particles are written, by new level, into the other; a particle whose step
// doubles (to level L0 - 1, not active) is appended to that level's current
// list. The plan of the next block flips the buffers of the active levels.
// List order is not significant: a target's sums do not depend on which
// targets share its group.
//
// Per block, three kernels in stream order:
//   k_bl_predict  tile kinds (active sets above 48) only: every particle
//                 predicted to t_next into the predicted arrays.
//   k_bl_eval     fixed grid; each workgroup takes (target group, source
//                 slice) units and writes slice sums. Small active sets
//                 predict their sources and targets on the fly from the state
//                 (a pass over all particles would cost more than their
//                 evaluation); the tile kinds read the predicted arrays.
//   k_bl_finish   compensated slice sums, corrector in place, list updates;
//                 the last workgroup plans the next block.
// Only the finishing workgroups (at most kFinGrid, fewer for small sets)
// synchronise through device-scope atomics: on this GPU such fences and
// atomics serialise across the device, so per-block atomics stay few.
// Descriptors are double-buffered by block parity: block b reads desc[b & 1]
// and its plan for b + 1 goes to desc[(b + 1) & 1], so no kernel of block b
// sees its own descriptor change.
#include <hip/hip_ext.h>

#include "eval_body.h"
#include "eval_mixed_body.h"
#include "steps_body.h"

namespace h6 {
namespace {

using namespace evalbody;
using namespace mixedbody;
using namespace stepbody;

constexpr int kSmall1Max = 16;   // active sets up to this size: one target per wave
constexpr int kTileBlock = 64;   // tile kinds: one-wave workgroups
constexpr int kTileIpl = 2;      // targets per lane of tile kind 0
constexpr int kTile1Max = 512;   // active sets up to this size: tile kind 2, one per lane
constexpr int kFinThreads = 512;
constexpr int kFinGrid = 128;    // finishing workgroups at most
constexpr int kScanThreads = 256;


template <typename T>
__device__ __forceinline__ T load_agent(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_agent(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned add_agent(unsigned *p, unsigned v) {
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Whether this workgroup is the last of `total` to arrive at `counter`
// (release of this workgroup's stores before, acquire of the others' after);
// the last one resets the counter. Every thread must call it.
__device__ __forceinline__ bool arrive_last(unsigned *counter, unsigned total) {
    __shared__ bool is_last;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned prev =
            __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        is_last = (prev == total - 1);
        if (is_last) store_agent(counter, 0u);
    }
    __syncthreads();
    if (is_last) __threadfence();
    return is_last;
}

__device__ __forceinline__ int32_t *level_list(const LoopArgs &A, int buf, int L) {
    return A.lists + ((int64_t)buf * A.nl + (L - A.lev_lo)) * (int64_t)A.n;
}

// The active levels' rank offsets and list buffers of a block, copied into
// LDS by every workgroup that maps ranks to particles.
struct RankTable {
    int L0, hi;
    unsigned long long sel;
    int off[kLevels];
};

// The descriptor fields a kernel of the loop reads, loaded together at its
// start (one round trip to memory instead of one per dependent branch);
// thread t < kLevels also takes off[t] and cnt[t]. Needs blockDim.x >= kLevels.
struct DescHead {
    int64_t t_next;
    unsigned long long sel;
    int n_act, split, slice_len, groups, kind, L0, lv_hi;
    int my_off, my_cnt;
};
__device__ __forceinline__ DescHead load_head(const LoopDesc *__restrict__ d) {
    DescHead h;
    h.t_next = d->t_next;
    h.sel = d->sel;
    h.n_act = d->n_act;
    h.split = d->split;
    h.slice_len = d->slice_len;
    h.groups = d->groups;
    h.kind = d->kind;
    h.L0 = d->L0;
    h.lv_hi = d->lv_hi;
    const int t = threadIdx.x < kLevels ? threadIdx.x : 0;
    h.my_off = d->off[t];
    h.my_cnt = d->cnt[t];
    return h;
}
// The rank table from a loaded head (every thread must call it).
__device__ __forceinline__ void rank_table_from(RankTable *rt, const DescHead &h) {
    if (threadIdx.x < kLevels) rt->off[threadIdx.x] = h.my_off;
    if (threadIdx.x == 0) {
        rt->L0 = h.L0;
        rt->hi = h.lv_hi;
        rt->sel = h.sel;
    }
    __syncthreads();
}

// Particle of active rank k: ranks run over the active levels from the
// highest down, level L holding ranks [off[L], off[L] + cnt[L]).
// Out-of-range indices (which the list bookkeeping never produces) are
// clamped and reported through the status flags instead of being used.
__device__ __forceinline__ int rank_to_particle(const LoopArgs &A, const RankTable *rt, int k) {
    int L = rt->L0;
    const int hi = rt->hi;
    while (L < hi && k < rt->off[L]) ++L;
    const int buf = (int)((rt->sel >> L) & 1ull);
    const int pos = k - rt->off[L];
    const bool pos_ok = pos >= 0 && pos < A.n && L >= A.lev_lo && L < A.lev_lo + A.nl;
    int id = level_list(A, pos_ok ? buf : 0, pos_ok ? L : A.lev_lo)[pos_ok ? pos : 0];
    if (!pos_ok || (unsigned)id >= (unsigned)A.n) {
        atomicOr(A.flags, kFlagLoop);
        id = 0;
    }
    return id;
}

// Source/target policies of the evaluation bodies; targets through the
// level lists. StateSrc predicts from the state to t_next on the fly,
// ListPredSrc reads the predicted arrays.
struct StateSrc {
    LoopArgs A;
    const RankTable *rt;
    int64_t t_next;
    __device__ __forceinline__ int target(int k) const { return rank_to_particle(A, rt, k); }
    template <int ORDER>
    __device__ __forceinline__ void get(int p, double *x, double *v, double *a, double *j) const {
        static_assert(ORDER == 2, "block steps evaluate a, j, s");
        predict_vals(A.st, p, (double)(t_next - A.st.t[p]) * kTick, x, v, a);
        j[0] = j[1] = j[2] = 0.0;
    }
    __device__ __forceinline__ double mass(int p) const { return A.st.m[p]; }
};

struct ListPredSrc {
    LoopArgs A;
    const RankTable *rt;
    __device__ __forceinline__ int target(int k) const { return rank_to_particle(A, rt, k); }
    template <int ORDER>
    __device__ __forceinline__ void get(int p, double *x, double *v, double *a, double *j) const {
        static_assert(ORDER == 2, "block steps evaluate a, j, s");
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[c] = A.pred.x[c][p];
            v[c] = A.pred.v[c][p];
            a[c] = A.pred.a[c][p];
            j[c] = 0.0;
        }
    }
    __device__ __forceinline__ double mass(int p) const { return A.st.m[p]; }
};

__device__ __forceinline__ int cdiv32(int a, int b) { return (a + b - 1) / b; }

// Evaluation shape for n_act targets (32-bit arithmetic: one thread runs
// it on the critical path). Source-parallel kinds (1: one target per wave,
// 3: two), which predict on the fly: slices of at least 256 sources (4 per
// lane), at most eval_grid waves in all. Tile kinds read the predicted
// arrays. Kind 2 (up to kTile1Max targets; 64 per one-wave workgroup, one
// per lane): the slice count from a small model of the time, below. Kind 0
// (128 targets per workgroup, two per lane): as many slices as fit one
// round of resident workgroups, down to one 64-source tile per slice; with
// few slices per group, the slice count that fills the last round best.
// The grid holds two waves per SIMD, which share its issue rate, so a round
// of units is one unit per SIMD. pc_pairs bounds split * n_act.
__device__ void launch_shape(LoopDesc *d, int n, int n_act, int eval_grid, unsigned pc_pairs) {
    int split, kind, groups;
    if (n_act <= kSmall2Max) {
        kind = n_act <= kSmall1Max ? 1 : 3;
        groups = kind == 1 ? n_act : cdiv32(n_act, 2);
        split = (n + 255) >> 8;
        const int fit = eval_grid / groups;
        split = split < fit ? split : fit;
    } else if (n_act <= kTile1Max) {
        // time in source rows of one unit, for r units per SIMD (r = 1..6):
        // rounds x slice length, a lone wave per SIMD issuing at about 3/4 of
        // the rate of two, plus the slice sums (72 bytes per slice and
        // target, written, read back and reduced: about 1/2400 row each)
        kind = 2;
        groups = cdiv32(n_act, kTileBlock);
        const int simds = eval_grid / 2;
        const int cap = (n + kTileBlock - 1) / kTileBlock;
        int64_t best_cost = INT64_MAX;
        split = 1;
        for (int r = 1; r <= 6; ++r) {
            int sp = r * simds / groups;
            sp = sp < 1 ? 1 : (sp > cap ? cap : sp);
            const int sl = cdiv32(cdiv32(n, sp), 64) * 64;
            sp = cdiv32(n, sl);
            const int units = groups * sp;
            int64_t cost = units <= simds ? (int64_t)sl + sl / 3
                                          : (int64_t)cdiv32(units, simds) * sl;
            cost += (int64_t)sp * n_act / 2400;
            if (cost < best_cost) {
                best_cost = cost;
                split = sp;
            }
        }
    } else {
        kind = 0;
        groups = cdiv32(n_act, kTileBlock * kTileIpl);
        split = eval_grid / groups;
        const int cap = (n + kTileBlock - 1) / kTileBlock;
        split = split < cap ? split : cap;
        if (split < 1) split = 1;
        if (split <= 16) {
            // few slices per group: the last round of units may leave SIMDs
            // idle. Take the slice count in [split, 4 split] with the least
            // rounds x slice length (ties: fewer slices).
            const int simds = eval_grid / 2;
            int best = split;
            int64_t best_cost = INT64_MAX;
            const int hi = 4 * split < cap ? 4 * split : cap;
            for (int sp = split; sp <= hi; ++sp) {
                const int sl = cdiv32(cdiv32(n, sp), 64) * 64;
                const int units = groups * cdiv32(n, sl);
                const int64_t cost = (int64_t)cdiv32(units, simds) * sl;  // ~n_act n / 2^17
                if (cost < best_cost) {
                    best_cost = cost;
                    best = sp;
                }
            }
            split = best;
        }
    }
    const unsigned pc = pc_pairs / (unsigned)n_act;
    if ((unsigned)split > pc) split = (int)pc;
    if (split < 1) split = 1;
    const int slice = cdiv32(cdiv32(n, split), 64) * 64;
    d->kind = kind;
    d->groups = groups;
    d->slice_len = slice;
    d->split = cdiv32(n, slice);
}

// Lanes per target in the finishing reduction: the power of two covering
// the slices, at most a wave; a wave sums 64 / seg targets at once.
__device__ __forceinline__ int fin_seg(int split) {
    int seg = 1;
    while (seg < split && seg < 64) seg <<= 1;
    return seg;
}
// Targets per finishing workgroup round and the number of finishing
// workgroups with work, for a block of n_act targets in `split` slices.
__device__ __forceinline__ int fin_per_round(int split) {
    return (64 / fin_seg(split)) * (kFinThreads / 64);
}
__device__ __forceinline__ int fin_workers(int n_act, int split) {
    const int w = cdiv32(n_act, fin_per_round(split));
    return w < kFinGrid ? w : kFinGrid;
}

// Plans the block after time t_cur into *d from the level counts cnt (in
// LDS; d->cnt is written by the caller), with blocks / particle_steps the
// totals so far: next block time, active levels and count, rank offsets,
// evaluation shape; n_act = 0 and done = 1 once t_next would pass t_end.
// One wave (all 64 lanes call it), lane L for level L: a wave minimum gives
// t_next, a ballot the occupied levels, a suffix scan the rank offsets.
__device__ void plan_block(const LoopArgs &A, LoopDesc *d, const int *cnt, int64_t t_cur,
                           uint64_t sel, int64_t blocks, int64_t psteps, int64_t seq_next) {
    static_assert(kLevels <= 64, "one lane per level");
    const int L = threadIdx.x & 63;
    const bool listed = L >= A.lev_lo && L < A.lev_lo + A.nl;
    const int c = listed ? cnt[L] : 0;
    // next multiple of 2^(40 - L) ticks after t_cur (t_cur >= 0)
    int64_t tn = INT64_MAX;
    if (c > 0) {
        const int sh = kTickBits - L;
        tn = ((t_cur >> sh) + 1) << sh;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const int64_t o = __shfl_xor(tn, off, 64);
        tn = o < tn ? o : tn;
    }
    const unsigned long long occ = __ballot(c > 0);
    const int lv_hi = occ ? 63 - __builtin_clzll(occ) : -1;
    const bool done = lv_hi < 0 || tn > A.t_end;
    int L0 = done ? lv_hi : kTickBits - __builtin_ctzll((unsigned long long)tn);
    if (!done && L0 < A.lev_lo) L0 = A.lev_lo;
    // ranks run over the active levels from the highest down
    const int mine = (!done && L >= L0) ? c : 0;
    int incl = mine;  // sum over levels >= L
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int o = __shfl_down(incl, off, 64);
        if (L + off < 64) incl += o;
    }
    const int n_act = __shfl(incl, 0, 64);
    if (!done && L >= L0 && L <= lv_hi) d->off[L] = incl - mine;
    if (L != 0) return;
    d->t_next = tn;
    d->lv_hi = lv_hi;
    d->sel = sel;
    d->invalid = 0;
    d->L0 = L0;
    d->done = done ? 1 : 0;
    if (!done) {
        launch_shape(d, A.n, n_act, A.eval_grid, A.pc_pairs);
        blocks += 1;
        psteps += n_act;
    }
    d->blocks = blocks;
    d->particle_steps = psteps;
    d->n_act = n_act;
    if (A.nact_log) A.nact_log[seq_next & A.log_mask] = n_act;
}

// List slots handed out in a block: the sizes of the rebuilt lists of the
// active levels and the count appended to level L0 - 1. Kept in LDS when a
// single workgroup finishes the block, in LoopScratch otherwise.
struct Tally {
    unsigned reb[kLevels];
    unsigned app;
};

// Level counts after block `cur` (cur_cnt: its counts, in LDS; the rebuilt
// lists of the active levels; the appended particles of level L0 - 1), then
// the plan of the next block into *dn. The whole workgroup, after every list
// update of the block: one thread per level gathers, one thread plans from
// LDS. solo: the tallies are this workgroup's (LDS), else the device's.
__device__ void plan_next(const LoopArgs &A, const LoopDesc *__restrict__ cur, const int *cur_cnt,
                          const Tally *solo, LoopDesc *dn, int64_t seq) {
    __shared__ int s_cnt[kLevels];
    LoopScratch *scr = A.scr;
    const int L0 = cur->L0;
    for (int L = threadIdx.x; L < kLevels; L += blockDim.x) {
        int c = cur_cnt[L];
        if (L >= A.lev_lo && L < A.lev_lo + A.nl) {
            if (L >= L0) {
                if (solo) {
                    c = (int)solo->reb[L];
                } else {
                    c = (int)load_agent(&scr->reb[L]);
                    store_agent(&scr->reb[L], 0u);
                }
            } else if (L == L0 - 1) {
                if (solo) {
                    c += (int)solo->app;
                } else {
                    c += (int)load_agent(&scr->app);
                    store_agent(&scr->app, 0u);
                }
            }
        }
        s_cnt[L] = c;
        dn->cnt[L] = c;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // list buffers flip for the active levels [max(L0, lev_lo), lev_lo + nl)
        const int lo = L0 > A.lev_lo ? L0 : A.lev_lo;
        const uint64_t flip = ((1ull << (A.lev_lo + A.nl)) - 1ull) & ~((1ull << lo) - 1ull);
        plan_block(A, dn, s_cnt, cur->t_next, cur->sel ^ flip, cur->blocks, cur->particle_steps,
                   seq + 1);
    }
}

__global__ __launch_bounds__(256) void k_bl_predict(LoopArgs A, int64_t seq) {
    const LoopDesc *__restrict__ d = A.desc + (seq & 1);
    if (d->n_act == 0 || (d->kind != 0 && d->kind != 2)) return;
    const int64_t tn = d->t_next;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += gridDim.x * blockDim.x)
        predict_one(A.st, i, (double)(tn - A.st.t[i]) * kTick, A.pred);
}

template <bool MIXED, bool SKIPSELF>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_bl_eval(
    LoopArgs A, int64_t seq) {
    const LoopDesc *__restrict__ d = A.desc + (seq & 1);
    const DescHead h = load_head(d);
    const int n_act = h.n_act;
    if (n_act == 0) return;
    const int split = h.split, slice_len = h.slice_len, groups = h.groups;
    const int kind = h.kind;
    // slice sums at partial[(k * 9 + c) * split + sl]: a target's slices are
    // contiguous for the finishing reduction
    OutPtrs out;
#pragma unroll
    for (int c = 0; c < kMaxOut; ++c) out.p[c] = c < 9 ? A.partial + (int64_t)c * split : nullptr;
    out.kstride = (int64_t)9 * split;
    const int64_t slice_stride = 1;
    const int units = groups * split;
    if ((int)blockIdx.x >= units) return;
    __shared__ RankTable rt;
    rank_table_from(&rt, h);
    if (kind == 0 || kind == 2) {
        const ListPredSrc S{A, &rt};
        for (int u = blockIdx.x; u < units; u += gridDim.x) {
            const int g = u / split, sl = u - g * split;
            if (kind == 0) {
                if constexpr (MIXED)
                    mixed_tile_body<kTileBlock, kTileIpl, SKIPSELF>(S, A.n, n_act, A.eps2,
                                                                    slice_len, out, slice_stride,
                                                                    g, sl);
                else
                    eval_tile_body<2, kTileBlock, kTileIpl, SKIPSELF>(S, A.n, n_act, A.eps2,
                                                                      slice_len, out,
                                                                      slice_stride, g, sl);
            } else {
                if constexpr (MIXED)
                    mixed_tile_body<kTileBlock, 1, SKIPSELF>(S, A.n, n_act, A.eps2, slice_len,
                                                             out, slice_stride, g, sl);
                else
                    eval_tile_body<2, kTileBlock, 1, SKIPSELF>(S, A.n, n_act, A.eps2, slice_len,
                                                               out, slice_stride, g, sl);
            }
        }
        return;
    }
    const StateSrc S{A, &rt, h.t_next};
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int g = u / split, sl = u - g * split;
        if (kind == 1) {
            if constexpr (MIXED)
                mixed_small_body<1, SKIPSELF>(S, A.n, n_act, A.eps2, slice_len, out, slice_stride,
                                              g, sl);
            else
                eval_small_body<1, SKIPSELF>(S, A.n, n_act, A.eps2, slice_len, out, slice_stride,
                                             g, sl);
        } else {
            if constexpr (MIXED)
                mixed_small_body<2, SKIPSELF>(S, A.n, n_act, A.eps2, slice_len, out, slice_stride,
                                              g, sl);
            else
                eval_small_body<2, SKIPSELF>(S, A.n, n_act, A.eps2, slice_len, out, slice_stride,
                                             g, sl);
        }
    }
}

// Workgroup-aggregated list insertion: one slot reservation per level per
// workgroup round, from the device counters, or from this workgroup's own
// tally (solo) when it finishes the block alone. cur_cnt: the block's
// level counts (LDS). Every thread calls it; valid marks the threads with a
// particle. Ends with a barrier.
__device__ void list_insert_wg(const LoopArgs &A, const RankTable *rt, const int *cur_cnt,
                               Tally *solo, bool valid, int id, int lev) {
    __shared__ unsigned lcount[kLevels];
    __shared__ unsigned lbase[kLevels];
    for (int L = threadIdx.x; L < kLevels; L += blockDim.x) lcount[L] = 0u;
    __syncthreads();
    unsigned rank = 0;
    if (valid) rank = atomicAdd(&lcount[lev], 1u);
    __syncthreads();
    const int L0 = rt->L0;
    for (int L = threadIdx.x; L < kLevels; L += blockDim.x) {
        const unsigned c = lcount[L];
        if (c > 0) {
            if (solo) {
                if (L >= L0) {
                    lbase[L] = solo->reb[L];
                    solo->reb[L] += c;
                } else {
                    lbase[L] = (unsigned)cur_cnt[L] + solo->app;
                    solo->app += c;
                }
            } else {
                lbase[L] = L >= L0 ? add_agent(&A.scr->reb[L], c)
                                   : (unsigned)cur_cnt[L] + add_agent(&A.scr->app, c);
            }
        }
    }
    __syncthreads();
    if (valid) {
        const int buf = (int)((rt->sel >> lev) & 1ull) ^ (lev >= L0 ? 1 : 0);
        const unsigned slot = lbase[lev] + rank;
        if (slot < (unsigned)A.n && lev >= A.lev_lo && lev < A.lev_lo + A.nl)
            level_list(A, buf, lev)[slot] = id;
        else
            atomicOr(A.flags, kFlagLoop);
    }
    __syncthreads();
}

// Neumaier step: s + comp += x.
__device__ __forceinline__ void neumaier(double &s, double &comp, double x) {
    const double t = s + x;
    comp += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
}

__global__ __launch_bounds__(kFinThreads) void k_bl_finish(LoopArgs A, int64_t seq) {
    const LoopDesc *__restrict__ d = A.desc + (seq & 1);
    LoopDesc *dn = A.desc + ((seq + 1) & 1);
    const DescHead h = load_head(d);
    const int n_act = h.n_act;
    if (n_act == 0) {
        // nothing due before t_end: carry the final descriptor forward
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            *dn = *d;
            if (A.nact_log) A.nact_log[(seq + 1) & A.log_mask] = 0;
        }
        return;
    }
    const int split = h.split;
    const int seg = fin_seg(split);
    const int per = fin_per_round(split);
    const int workers = fin_workers(n_act, split);
    if ((int)blockIdx.x >= workers) return;
    const int64_t tn = h.t_next;
    const bool solo = workers == 1;  // no other workgroup: tallies in LDS, no device atomics
    __shared__ double fs[kFinThreads * 9];
    __shared__ RankTable rt;
    __shared__ int cur_cnt[kLevels];
    __shared__ Tally tally;
    if (threadIdx.x < kLevels) {
        cur_cnt[threadIdx.x] = h.my_cnt;
        tally.reb[threadIdx.x] = 0u;
    }
    if (threadIdx.x == 0) tally.app = 0u;
    rank_table_from(&rt, h);  // ends with a barrier
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    for (int k0 = blockIdx.x * per; k0 < n_act; k0 += workers * per) {
        const int nt = n_act - k0 < per ? n_act - k0 : per;
        const bool valid = tid < nt;
        int id = 0, lev = 0;
        OldState old{};
        const bool reducer = w * (64 / seg) < nt;  // waves holding a target of the round
        // seg lanes per target (contiguous slices: coalesced loads), the nine
        // components' loads of four passes issued together, then a fixed
        // butterfly within the segment
        const double *__restrict__ part = A.partial;
        const int r = w * (64 / seg) + lane / seg;  // target of this lane in the round
        const int o = lane & (seg - 1);
        const bool has = reducer && r < nt;
        const int64_t base = (int64_t)(k0 + (has ? r : 0)) * 9 * split;
        double x[4][9];
        auto load_slices = [&](int sl0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int sl = sl0 + q * seg + o;
                const bool in = has && sl < split;
#pragma unroll
                for (int c = 0; c < 9; ++c) x[q][c] = in ? part[base + c * split + sl] : 0.0;
            }
        };
        // the first slices, then the particle and its old state (list, then
        // state: two dependent loads), all in flight together
        if (reducer) load_slices(0);
        if (valid) {
            id = rank_to_particle(A, &rt, k0 + tid);
            old = load_old<false>(A.st, id);
        }
        if (reducer) {
            double s[9], comp[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) s[c] = comp[c] = 0.0;
            for (int sl0 = 0; sl0 < split; sl0 += 4 * seg) {
                if (sl0 != 0) load_slices(sl0);
#pragma unroll
                for (int q = 0; q < 4; ++q)
#pragma unroll
                    for (int c = 0; c < 9; ++c) neumaier(s[c], comp[c], x[q][c]);
            }
            seg_comp_reduce_n<9>(s, comp, seg);  // totals in the segment's last lane
#pragma unroll
            for (int c = 0; c < 9; ++c)
                if (has && o == seg - 1) fs[r * 9 + c] = s[c] + comp[c];
        }
        __syncthreads();
        if (valid) {
            double x1[3], v1[3], c1[3], f[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) f[c] = fs[tid * 9 + c];
            correct_from<false>(old, f, f + 3, f + 6, tn, 0.0, A.eta6, A.lev_min, A.lev_max,
                                A.flags, x1, v1, c1, &lev);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                A.st.x[c][id] = x1[c];
                A.st.v[c][id] = v1[c];
                A.st.a[c][id] = f[c];
                A.st.j[c][id] = f[3 + c];
                A.st.s[c][id] = f[6 + c];
                A.st.c[c][id] = c1[c];
            }
            A.st.t[id] = tn;
            A.st.dt[id] = (int64_t)1 << (kTickBits - lev);
        }
        list_insert_wg(A, &rt, cur_cnt, solo ? &tally : nullptr, valid, id, lev);
        // (ends with a barrier: fs reusable)
    }
    if (solo) {
        plan_next(A, d, cur_cnt, &tally, dn, seq);
        return;
    }
    if (!arrive_last(&A.scr->done_fin, (unsigned)workers)) return;
    plan_next(A, d, cur_cnt, nullptr, dn, seq);
}

// ---------------------------------------------------------------- set-up

__global__ void k_bl_setup_init(LoopArgs A) {
    LoopScratch *scr = A.scr;
    for (int i = threadIdx.x; i < kLevels; i += blockDim.x) scr->reb[i] = 0u;
    if (threadIdx.x == 0) {
        scr->done_fin = scr->app = scr->bad = 0u;
        scr->t_max = 0ull;
        scr->due_min = ~0ull;
    }
}

__device__ __forceinline__ unsigned long long wg_reduce_u64(unsigned long long v, bool take_max) {
    __shared__ unsigned long long part[kScanThreads / 64];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const unsigned long long o = __shfl_xor(v, off, 64);
        v = take_max ? (o > v ? o : v) : (o < v ? o : v);
    }
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long r = part[0];
    for (int q = 1; q < kScanThreads / 64; ++q)
        r = take_max ? (part[q] > r ? part[q] : r) : (part[q] < r ? part[q] : r);
    __syncthreads();
    return r;
}

// Checks that every particle sits on the block grid (step a power of two
// within the run's levels, time a multiple of it), finds the latest time
// and the earliest due time, and fills list buffer 0 by level.
__global__ __launch_bounds__(kScanThreads) void k_bl_setup_scan(LoopArgs A) {
    const int i = blockIdx.x * kScanThreads + threadIdx.x;
    const bool in = i < A.n;
    int64_t t = 0, dt = 1;
    if (in) {
        t = A.st.t[i];
        dt = A.st.dt[i];
    }
    bool ok = dt > 0 && (dt & (dt - 1)) == 0 && dt <= ((int64_t)1 << kTickBits) && t >= 0 &&
              t <= ((int64_t)1 << 61) && t % dt == 0;
    const int lev = ok ? level_of_ticks(dt) : -1;
    ok = ok && lev >= A.lev_lo && lev < A.lev_lo + A.nl;
    const bool bad = in && !ok;
    const unsigned nbad = (unsigned)__popcll(__ballot(bad));
    if ((threadIdx.x & 63) == 0 && nbad) add_agent(&A.scr->bad, nbad);
    const bool good = in && ok;
    const unsigned long long tmax = wg_reduce_u64(good ? (unsigned long long)t : 0ull, true);
    const unsigned long long dmin =
        wg_reduce_u64(good ? (unsigned long long)(t + dt) : ~0ull, false);
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_max(&A.scr->t_max, tmax, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_min(&A.scr->due_min, dmin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // fill: buffer 0, slots from the rebuild counters
    __shared__ unsigned lcount[kLevels];
    __shared__ unsigned lbase[kLevels];
    for (int L = threadIdx.x; L < kLevels; L += blockDim.x) lcount[L] = 0u;
    __syncthreads();
    unsigned rank = 0;
    if (good) rank = atomicAdd(&lcount[lev], 1u);
    __syncthreads();
    for (int L = threadIdx.x; L < kLevels; L += blockDim.x)
        if (lcount[L] > 0) lbase[L] = add_agent(&A.scr->reb[L], lcount[L]);
    __syncthreads();
    if (good) level_list(A, 0, lev)[lbase[lev] + rank] = i;
}

// Level counts from the fill, then the plan of block 0 into desc[0]; a
// state off the block grid is reported as invalid (and done).
__global__ void k_bl_setup_plan(LoopArgs A) {
    __shared__ int s_cnt[kLevels];
    LoopScratch *scr = A.scr;
    LoopDesc *d = A.desc;
    const unsigned long long tmax = scr->t_max, dmin = scr->due_min;
    const bool invalid = scr->bad != 0u || dmin <= tmax;
    for (int L = threadIdx.x; L < kLevels; L += blockDim.x) {
        const int c = invalid ? 0 : (int)scr->reb[L];
        s_cnt[L] = c;
        d->cnt[L] = c;
        scr->reb[L] = 0u;
    }
    __syncthreads();
    if (invalid) {
        if (threadIdx.x != 0) return;
        scr->bad = 0u;
        d->sel = 0ull;
        d->blocks = 0;
        d->particle_steps = 0;
        d->invalid = 1;
        d->n_act = 0;
        d->done = 1;
        d->t_next = 0;
        if (A.nact_log) A.nact_log[0] = 0;
        return;
    }
    if (threadIdx.x == 0) scr->bad = 0u;
    if (threadIdx.x < 64) plan_block(A, d, s_cnt, (int64_t)tmax, 0ull, 0, 0, 0);
}

}  // namespace

int bl_eval_grid(h6_ctx ctx) { return ctx->n_cu * 8; }  // one round of resident tile workgroups

int64_t bl_list_ints(int64_t n, int nl) { return 2 * (int64_t)nl * n; }

hipError_t bl_setup(h6_ctx ctx, const LoopArgs &A) {
    hipLaunchKernelGGL(k_bl_setup_init, dim3(1), dim3(64), 0, ctx->stream, A);
    hipLaunchKernelGGL(k_bl_setup_scan, dim3((A.n + kScanThreads - 1) / kScanThreads),
                       dim3(kScanThreads), 0, ctx->stream, A);
    hipLaunchKernelGGL(k_bl_setup_plan, dim3(1), dim3(64), 0, ctx->stream, A);
    return hipGetLastError();
}

hipError_t bl_enqueue_block(h6_ctx ctx, const LoopArgs &A, int precision, int64_t seq) {
    const int pgrid = ctx->n_cu > 1 ? ctx->n_cu / 2 : 1;
    hipLaunchKernelGGL(k_bl_predict, dim3(pgrid), dim3(256), 0, ctx->stream, A, seq);
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (ctx->prof) {
        hipError_t pe = prof_events(ctx, &ev0, &ev1);
        if (pe != hipSuccess) return pe;
    }
    const bool skip = self_pair_masked(A.eps2, precision);
    const bool mixed = precision == H6_MIXED;
    // with the measurement hook on, the events are those of the dispatch
    // itself (no separate marker packets in the stream)
#define H6_BL_EVAL(M, S)                                                                         \
    hipExtLaunchKernelGGL((k_bl_eval<M, S>), dim3(A.eval_grid), dim3(64), 0, ctx->stream, ev0, \
                          ev1, 0u, A, seq)
    if (mixed) {
        if (skip) H6_BL_EVAL(true, true); else H6_BL_EVAL(true, false);
    } else {
        if (skip) H6_BL_EVAL(false, true); else H6_BL_EVAL(false, false);
    }
#undef H6_BL_EVAL
    if (ctx->prof) {
        hipError_t pe = hipGetLastError();
        if (pe != hipSuccess) return pe;
        pe = prof_push_seq(ctx, ev0, ev1, precision, seq);
        if (pe != hipSuccess) return pe;
    }
    hipLaunchKernelGGL(k_bl_finish, dim3(kFinGrid), dim3(kFinThreads), 0, ctx->stream, A, seq);
    return hipGetLastError();
}

}  // namespace h6
