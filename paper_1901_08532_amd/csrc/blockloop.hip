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
// Per block, two kernels in stream order:
//   k_bl_eval     fixed grid; each workgroup takes (target group, source
//                 slice) units and writes slice sums, reading sources and
//                 targets from the predicted arrays.
//   k_bl_finish   compensated slice sums, corrector in place, list updates,
//                 and the prediction of every particle to the next block's
//                 likely time (the highest occupied level is always active,
//                 so unless a correction changes that level the next block
//                 comes one of its steps later); the last workgroup plans
//                 the next block. A wrong guess costs one prediction slot
//                 (the same two kernels: an empty evaluation, then a full
//                 prediction to the planned time). Measured on this GPU,
//                 predicting each source in every evaluation wave that
//                 reads it is slower than this, even for one or two active
//                 particles at N = 65536.
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
constexpr int kFinGrid = 128;    // finishing workgroups with targets at most
constexpr int kFinLaunch = 2 * kFinGrid;  // finishing kernel grid: the rest only predict
constexpr int kFinSplitNarrow = 64;  // slices up to this: threads over targets; more: a wave each
constexpr int kFinGroups = 7;    // wave-per-target reduction: lanes per component (9 x 7 of 64)
constexpr int kStash = 2048;     // corrected particles a finishing workgroup holds for insertion
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
    int64_t t_next, blocks, particle_steps;
    unsigned long long sel;
    int n_act, split, slice_len, groups, kind, L0, lv_hi, pred_ok;
    int my_off, my_cnt;
};
__device__ __forceinline__ DescHead load_head(const LoopDesc *__restrict__ d) {
    DescHead h;
    h.t_next = d->t_next;
    h.blocks = d->blocks;
    h.particle_steps = d->particle_steps;
    h.sel = d->sel;
    h.n_act = d->n_act;
    h.split = d->split;
    h.slice_len = d->slice_len;
    h.groups = d->groups;
    h.kind = d->kind;
    h.L0 = d->L0;
    h.lv_hi = d->lv_hi;
    h.pred_ok = d->pred_ok;
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

// Source/target policy of the evaluation bodies: targets through the level
// lists, sources and targets from the predicted arrays.
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

// Threads per target in the narrow finishing reduction (split <=
// kFinSplitNarrow): the power of two covering the slices in fours.
__device__ __forceinline__ int fin_seg(int split) {
    int seg = 1;
    while (4 * seg < split) seg <<= 1;
    return seg;
}
// Waves per target in the wide finishing reduction (split > kFinSplitNarrow):
// the power of two covering the slices in 256s, at most the workgroup's 8;
// a block that fits one round with waves to spare spreads each target's
// slices over more waves (shorter per-lane sum chains, down to 4 slices
// per lane).
__device__ __forceinline__ int fin_wpt(int split, int n_act) {
    constexpr int kWaves = kFinThreads / 64;
    int w = 1;
    while (256 * w < split && w < kWaves) w <<= 1;
    while (w < kWaves && kWaves / (2 * w) >= n_act && split >= 4 * kFinGroups * 2 * w) w <<= 1;
    return w;
}
// Targets per finishing workgroup round: kFinThreads / seg with few slices,
// 8 / fin_wpt with more.
__device__ __forceinline__ int fin_per_round(int split, int n_act) {
    return split > kFinSplitNarrow ? kFinThreads / 64 / fin_wpt(split, n_act)
                                   : kFinThreads / fin_seg(split);
}
// Evaluation shape for n_act targets, chosen by one wave (every lane calls
// it, lane 0 writes *d; every lane gets the slice count back).
// Source-parallel kinds (1: one target per wave, 3: two): slices of at least
// 256 sources, at most eval_grid waves in all (the mixed form one target
// per wave only, which keeps its kernel within four waves' registers). Tile kinds: kind 2 (up to kTile1Max targets) has 64 targets per one-wave
// workgroup (one per lane), kind 0 128 (two per lane). The grid holds two
// waves per SIMD (the mixed form four, priced as two per half SIMD), which
// share its issue rate, so a round of units is one unit per SIMD. For a tile kind lanes r - 1 and r + 7 (r = 1..8) price
// the shape whose units fill r rounds (the first with its slice count
// rounded as below): the time in source rows of one unit is rounds
// x slice length (a lone unit per SIMD issuing at about 3/4 of the rate of
// two), plus the slice sums (72 bytes per slice and target, written, read
// back and reduced: about 1/2400 row of a 64-target unit each); the
// cheapest shape wins, ties going to fewer slices. pc_pairs bounds
// split * n_act. Slice counts from 8 up are rounded up to multiples of 8
// (empty trailing slices) where the grid and pc_pairs allow, and for the
// tile kinds where the price is within 2%: unit g * split + sl then runs on XCD
// sl mod 8 for every target group g, so each XCD reads one eighth of the
// sources.
__device__ int launch_shape(LoopDesc *d, int n, int n_act, int eval_grid, bool one_small,
                            unsigned pc_pairs) {
    const int lane = threadIdx.x & 63;
    const int pc = (int)(pc_pairs / (unsigned)n_act) > 0 ? (int)(pc_pairs / (unsigned)n_act) : 1;
    int split, kind, groups, slice;
    if (n_act <= kSmall2Max) {
        kind = n_act <= kSmall1Max || one_small ? 1 : 3;
        groups = kind == 1 ? n_act : cdiv32(n_act, 2);
        split = (n + 255) >> 8;
        const int fit = eval_grid / groups;
        split = split < fit ? split : fit;
        split = split < pc ? split : pc;
        if (split < 1) split = 1;
        slice = cdiv32(cdiv32(n, split), 64) * 64;
        split = cdiv32(n, slice);
        const int sp8 = (split + 7) & ~7;  // whole XCD classes (below)
        if (split >= 8 && sp8 <= fit && sp8 <= pc) split = sp8;
    } else {
        const bool one = n_act <= kTile1Max;
        kind = one ? 2 : 0;
        const int tb = one ? kTileBlock : kTileBlock * kTileIpl;  // targets per unit
        groups = cdiv32(n_act, tb);
        const int simds = eval_grid / 2;
        const int cap = cdiv32(n, 64) < pc ? cdiv32(n, 64) : pc;
        int sp = 1, sl = 64;
        // prices in float (32-bit arithmetic only: 64-bit divisions expand to
        // long sequences on this GPU, and the planner is on every block's
        // critical path); the same inputs give the same shape on every run
        float cost = 3.0e38f;
        if (lane < 16) {
            const int r = (lane & 7) + 1;
            sp = r * simds / groups;
            sp = sp < 1 ? 1 : (sp > cap ? cap : sp);
            sl = cdiv32(cdiv32(n, sp), 64) * 64;
            sp = cdiv32(n, sl);
            // lanes 0..7: a multiple of 8 slices (the last ones empty) when
            // the partial buffer allows; lanes 8..15 the same shapes unrounded
            const int sp8 = (sp + 7) & ~7;
            if (lane < 8 && sp >= 8 && sp8 <= pc) sp = sp8;
            const int units = groups * sp;  // below 2^27 (pc_pairs bounds sp * n_act)
            const float ipl = (float)(tb / kTileBlock);
            cost = units <= simds ? (float)sl * (4.0f / 3.0f)
                                  : ceilf((float)units / (float)simds) * (float)sl;
            cost += (float)sp * (float)n_act / (2400.0f * ipl);
            // the finishing kernel's rounds, each about 10 us (42 rows of a
            // 64-target unit)
            const float fr =
                ceilf(ceilf((float)n_act / (float)fin_per_round(sp, n_act)) / (float)kFinGrid);
            cost += fr * 42.0f / ipl;
            // XCD-aligned slices win within 2% (fewer source re-reads)
            if (lane < 8 && (sp & 7) == 0) cost *= 0.98f;
        }
        // the cheapest of the 16 candidates (lanes 0..15, one DPP row): the
        // costs are positive, so their bit patterns order like the values;
        // the low 4 bits carry the lane, so ties go to the lowest lane (the
        // candidates' slice counts grow with r: the fewest slices, rounded
        // ones first)
        const unsigned key = (__float_as_uint(cost) & ~15u) | (unsigned)(lane & 15);
        const int win = (int)(__builtin_amdgcn_readfirstlane(row_min_u32(key)) & 15u);
        split = __builtin_amdgcn_readlane(sp, win);
        slice = __builtin_amdgcn_readlane(sl, win);
    }
    if (lane == 0) {
        d->kind = kind;
        d->groups = groups;
        d->slice_len = slice;
        d->split = split;
    }
    return split;
}

__device__ __forceinline__ int fin_workers(int n_act, int split) {
    const int w = cdiv32(n_act, fin_per_round(split, n_act));
    return w < kFinGrid ? w : kFinGrid;
}

// Plans the block after time t_cur into *d from the level counts cnt (in
// LDS; d->cnt is written by the caller), with blocks / particle_steps the
// totals so far: next block time, active levels and count, rank offsets,
// evaluation shape; n_act = 0 and done = 1 once t_next would pass t_end.
// t_spec: the time every particle was predicted to (-1: none), which makes
// the plan's pred_ok.
// One wave (all 64 lanes call it), lane L for level L: a ballot gives the
// occupied levels and t_next, per-lane sums over LDS the rank offsets.
__device__ void plan_block(const LoopArgs &A, LoopDesc *d, const int *cnt, int64_t t_cur,
                           uint64_t sel, int64_t blocks, int64_t psteps, int64_t seq_next,
                           int64_t t_spec) {
    static_assert(kLevels <= 64, "one lane per level");
    const int L = threadIdx.x & 63;
    const bool listed = L >= A.lev_lo && L < A.lev_lo + A.nl;
    const int c = listed ? cnt[L] : 0;
    const unsigned long long occ = __ballot(c > 0);
    const int lv_hi = occ ? 63 - __builtin_clzll(occ) : -1;
    // the earliest of the occupied levels' next due times after t_cur
    // (t_cur >= 0): that of the highest level, the next multiple of its step
    // 2^(40 - lv_hi) ticks -- every coarser step is a multiple of it, so a
    // coarser level's next multiple is never earlier
    int64_t tn = INT64_MAX;
    if (lv_hi >= 0) {
        const int sh = kTickBits - lv_hi;
        tn = ((t_cur >> sh) + 1) << sh;
    }
    const bool done = lv_hi < 0 || tn > A.t_end;
    int L0 = done ? lv_hi : kTickBits - __builtin_ctzll((unsigned long long)tn);
    if (!done && L0 < A.lev_lo) L0 = A.lev_lo;
    // ranks run over the active levels from the highest down: lane L of an
    // active level sums the counts of the levels L .. lv_hi (all listed)
    const bool act = !done && L >= L0 && L <= lv_hi;
    int incl = 0;
    if (act)
        for (int l = L; l <= lv_hi; ++l) incl += cnt[l];
    const int n_act = done ? 0 : __builtin_amdgcn_readlane(incl, L0);
    if (act) d->off[L] = incl - c;
    const int split =
        done ? 0
             : launch_shape(d, A.n, n_act, A.eval_grid, A.one_target_small != 0,
                            A.pc_pairs);  // the whole wave
    if (L != 0) return;
    d->t_next = tn;
    d->lv_hi = lv_hi;
    d->sel = sel;
    d->invalid = 0;
    d->L0 = L0;
    d->done = done ? 1 : 0;
    if (!done) {
        blocks += 1;
        psteps += n_act;
    }
    d->blocks = blocks;
    d->particle_steps = psteps;
    d->n_act = n_act;
    // the finishing kernel predicted every particle to t_spec: right unless
    // the highest occupied level changed; else the next slot predicts
    const bool pred_ok = !done && tn == t_spec;
    d->pred_ok = pred_ok ? 1 : 0;
    if (A.nact_log) {
        int32_t *e = A.nact_log + 2 * (seq_next & A.log_mask);
        e[0] = n_act;
        e[1] = done ? 0 : (pred_ok ? split : -1);
    }
}

// List slots handed out in a block: the sizes of the rebuilt lists of the
// active levels and the count appended to level L0 - 1. Kept in LDS when a
// single workgroup finishes the block, in LoopScratch otherwise.
struct Tally {
    unsigned reb[kLevels];
    unsigned app;
};

// Level counts after block `cur` (its descriptor head as loaded at the
// kernel's start; cur_cnt: its counts, in LDS; the rebuilt
// lists of the active levels; the appended particles of level L0 - 1), then
// the plan of the next block into *dn. The whole workgroup, after every list
// update of the block: one thread per level gathers, one wave plans from
// LDS. solo: the tallies are this workgroup's (LDS), else the device's.
__device__ void plan_next(const LoopArgs &A, const DescHead &cur, const int *cur_cnt,
                          const Tally *solo, LoopDesc *dn, int64_t seq, int64_t t_spec) {
    __shared__ int s_cnt[kLevels];
    LoopScratch *scr = A.scr;
    const int L0 = cur.L0;
    for (int L = threadIdx.x; L < kLevels; L += blockDim.x) {
        int c = cur_cnt[L];
        if (L >= A.lev_lo && L < A.lev_lo + A.nl) {
            if (L >= L0) {
                if (solo) {
                    c = (int)solo->reb[L];
                } else {
                    c = (int)load_agent(&scr->reb[L][0]);
                    store_agent(&scr->reb[L][0], 0u);
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
        plan_block(A, dn, s_cnt, cur.t_next, cur.sel ^ flip, cur.blocks, cur.particle_steps,
                   seq + 1, t_spec);
    }
}

// Storage slot of slice sl of target group g in the wide slice-sum layout
// ([k][c][slot]): the group's slices ordered by the XCD that computes them,
// then by slice. Unit u = g * split + sl runs on workgroup u mod grid, which
// the dispatcher places on XCD u mod 8 (round robin; the grid is a multiple
// of 8), so consecutive slots -- the lines holding a target's slice sums --
// are written through one XCD's L2 instead of partially through all eight.
// A bijection of [0, split) for every g.
__device__ __forceinline__ int xcd_slot(int g, int sl, int split) {
    const int base = (int)(((int64_t)g * split) & 7);  // XCD of the group's slice 0
    const int x = (base + sl) & 7;
    int before = 0;  // the group's slices on lower XCDs
    for (int y = 0; y < x; ++y) {
        const int s0 = (y - base) & 7;  // the group's first slice on XCD y
        before += s0 < split ? (split - 1 - s0) / 8 + 1 : 0;
    }
    return before + (sl - ((x - base) & 7)) / 8;
}

template <bool MIXED, bool SKIPSELF>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(MIXED ? 4 : 2))) void k_bl_eval(
    LoopArgs A, int64_t seq) {
    const LoopDesc *__restrict__ d = A.desc + (seq & 1);
    const DescHead h = load_head(d);
    const int n_act = h.n_act;
    if (n_act == 0 || !h.pred_ok) return;  // nothing due, or a prediction slot
    const int split = h.split, slice_len = h.slice_len, groups = h.groups;
    const int kind = h.kind;
    // slice sums: with few slices (the finishing kernel gives each target a
    // thread) at partial[(sl * 9 + c) * n_act + k], consecutive targets
    // adjacent; with more (a wave per target) at partial[(k * 9 + c) * split
    // + xcd_slot(g, sl)], a target's slices adjacent
    const bool narrow = split <= kFinSplitNarrow;
    OutPtrs out;
#pragma unroll
    for (int c = 0; c < kMaxOut; ++c)
        out.p[c] = c < 9 ? A.partial + (int64_t)c * (narrow ? n_act : split) : nullptr;
    out.kstride = narrow ? 1 : (int64_t)9 * split;
    const int64_t slice_stride = narrow ? (int64_t)9 * n_act : 1;
    // the output of unit (g, sl): the bodies write component c of target k
    // at p[c][sl * slice_stride + k * kstride]; the wide layout's slot shift
    // goes into the pointers
    auto out_of = [&](int g, int sl) {
        OutPtrs o = out;
        if (!narrow) {
            const int shift = xcd_slot(g, sl, split) - sl;
#pragma unroll
            for (int c = 0; c < 9; ++c) o.p[c] += shift;
        }
        return o;
    };
    const int units = groups * split;
    if ((int)blockIdx.x >= units) return;
    __shared__ RankTable rt;
    rank_table_from(&rt, h);
    // one workgroup-memory pool for the bodies (a tile, or the small sets'
    // final reduction over 9 * 2 values per lane)
    constexpr int kPool2 = 64 * 9;  // double2
    static_assert(kPool2 >= kTileBlock * Traits<2>::NREC, "FP64 tile fits the pool");
    static_assert(kPool2 * sizeof(double2) >= kTileBlock * sizeof(RecMixed), "mixed tile fits");
    __shared__ double2 pool[kPool2];
    double2 *tile = pool;
    RecMixed *tile_m = reinterpret_cast<RecMixed *>(pool);
    double *red = reinterpret_cast<double *>(pool);
    if (kind == 0 || kind == 2) {
        const ListPredSrc S{A, &rt};
        for (int u = blockIdx.x; u < units; u += gridDim.x) {
            const int g = u / split, sl = u - g * split;
            const OutPtrs o = out_of(g, sl);
            if (kind == 0) {
                if constexpr (MIXED)
                    mixed_tile_body<kTileBlock, kTileIpl, SKIPSELF>(S, A.n, n_act, A.eps2,
                                                                    slice_len, o, slice_stride,
                                                                    g, sl, tile_m);
                else
                    eval_tile_body<2, kTileBlock, kTileIpl, SKIPSELF, false>(
                        S, A.n, n_act, A.eps2, slice_len, o, slice_stride, g, sl, tile);
            } else {
                if constexpr (MIXED)
                    mixed_tile_body<kTileBlock, 1, SKIPSELF>(S, A.n, n_act, A.eps2, slice_len,
                                                             o, slice_stride, g, sl, tile_m);
                else
                    eval_tile_body<2, kTileBlock, 1, SKIPSELF, true>(
                        S, A.n, n_act, A.eps2, slice_len, o, slice_stride, g, sl, tile);
            }
        }
        return;
    }
    {
        const ListPredSrc S{A, &rt};
        for (int u = blockIdx.x; u < units; u += gridDim.x) {
            const int g = u / split, sl = u - g * split;
            const OutPtrs o = out_of(g, sl);
            if (kind == 1) {
                // mixed: two sources per lane in flight, so that the kernel
                // fits the registers of four waves per SIMD
                if constexpr (MIXED)
                    mixed_small_body<1, SKIPSELF, 2>(S, A.n, n_act, A.eps2, slice_len, o,
                                                     slice_stride, g, sl, red);
                else
                    eval_small_body<1, SKIPSELF>(S, A.n, n_act, A.eps2, slice_len, o,
                                                 slice_stride, g, sl, red);
            } else {
                // two targets per wave: FP64 only (the mixed plan takes one)
                if constexpr (MIXED) {
                    if (threadIdx.x == 0) atomicOr(A.flags, kFlagLoop);
                } else {
                    eval_small_body<2, SKIPSELF>(S, A.n, n_act, A.eps2, slice_len, o,
                                                 slice_stride, g, sl, red);
                }
            }
        }
    }
}

// List insertion of the particles a finishing workgroup corrected (held in
// LDS, ids and new levels): one slot reservation per level for all of them,
// from the device counters (a line each), or from this workgroup's own
// tally (solo) when it finishes the block alone. cur_cnt: the block's level
// counts (LDS). Every thread calls it; it starts and ends with a barrier.
__device__ void list_insert_stash(const LoopArgs &A, const RankTable *rt, const int *cur_cnt,
                                  Tally *solo, const int32_t *st_id, const uint8_t *st_lev,
                                  int nst) {
    __shared__ unsigned lcount[kLevels];
    __shared__ unsigned lbase[kLevels];
    constexpr int kPer = kStash / kFinThreads;
    __syncthreads();
    for (int L = threadIdx.x; L < kLevels; L += blockDim.x) lcount[L] = 0u;
    __syncthreads();
    unsigned rank[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int e = q * kFinThreads + threadIdx.x;
        rank[q] = e < nst ? atomicAdd(&lcount[st_lev[e]], 1u) : 0u;
    }
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
                lbase[L] = L >= L0 ? add_agent(&A.scr->reb[L][0], c)
                                   : (unsigned)cur_cnt[L] + add_agent(&A.scr->app, c);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int e = q * kFinThreads + threadIdx.x;
        if (e < nst) {
            const int lev = st_lev[e];
            const int buf = (int)((rt->sel >> lev) & 1ull) ^ (lev >= L0 ? 1 : 0);
            const unsigned slot = lbase[lev] + rank[q];
            if (slot < (unsigned)A.n && lev >= A.lev_lo && lev < A.lev_lo + A.nl)
                level_list(A, buf, lev)[slot] = st_id[e];
            else
                atomicOr(A.flags, kFlagLoop);
        }
    }
    __syncthreads();
}

// Wide finishing reduction of one round (targets k0 .. k0 + nt - 1, nt <=
// 8 / WPT): waves WPT r .. WPT r + WPT - 1 take target k0 + r; lane (c, g)
// of the p-th of them sums slices g', g' + G, ... of component c (g' = 7 p
// + g, G = 7 WPT) into a compensated pair, and lane c of the first wave
// merges the 7 WPT pairs in order into fs[r * 9 + c]. particle() issues the
// correcting threads' own loads after the first slices'. Every thread
// calls it (it contains a barrier).
template <int WPT, class PARTICLE>
__device__ __forceinline__ void fin_wide_sums(const double *__restrict__ part, int k0, int nt,
                                              int split, double2 *gsum, double *fs,
                                              PARTICLE particle) {
    constexpr int G = kFinGroups * WPT;
    constexpr int U = 19;  // two batches hold the 37 slices per lane of split <= 256 * WPT
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int r = w / WPT, pw = w % WPT;
    const int c = lane / kFinGroups, g = lane % kFinGroups;
    const int gg = pw * kFinGroups + g;
    const bool has = r < nt && c < 9;
    const double *__restrict__ pc =
        part + ((int64_t)(k0 + (has ? r : 0)) * 9 + (has ? c : 0)) * split + gg;
    const int nq = has && gg < split ? (split - gg + G - 1) / G : 0;
    double xa[U], xb[U];
    auto load = [&](double *x, int i0) {
#pragma unroll
        for (int u = 0; u < U; ++u) x[u] = i0 + u < nq ? pc[G * (i0 + u)] : 0.0;
    };
    // two batches of slices and the particle's list entry in flight
    // together, then its old state (dependent on the list entry) while the
    // batches are summed: two memory round trips in all
    const int nq_max = (split + G - 1) / G;
    load(xa, 0);
    if (U < nq_max) load(xb, U);
    particle();
    double hs = 0.0, hc = 0.0;
    for (int i0 = 0; i0 < nq_max; i0 += 2 * U) {
        if (i0 > 0) {
            load(xa, i0);
            if (i0 + U < nq_max) load(xb, i0 + U);
        }
#pragma unroll
        for (int u = 0; u < U; ++u) two_sum_into(hs, hc, xa[u]);
        if (i0 + U >= nq_max) break;
#pragma unroll
        for (int u = 0; u < U; ++u) two_sum_into(hs, hc, xb[u]);
    }
    gsum[tid] = make_double2(hs, hc);
    __syncthreads();
    if (pw == 0 && r < nt && lane < 9) {
        double ts = 0.0, tc = 0.0;
#pragma unroll
        for (int q = 0; q < WPT; ++q)
#pragma unroll
            for (int gq = 0; gq < kFinGroups; ++gq) {
                const double2 e = gsum[(w + q) * 64 + lane * kFinGroups + gq];
                comp_merge(ts, tc, e.x, e.y);
            }
        fs[r * 9 + lane] = ts + tc;
    }
}

// The targets of one finishing workgroup (rounds of per targets): slice
// sums, corrector, prediction of the corrected particle to t_spec, list
// insertion; then the plan of the next block by the last workgroup.
__device__ __forceinline__ void finish_targets(const LoopArgs &A, const DescHead &h,
                                               const LoopDesc *__restrict__ d, LoopDesc *dn,
                                               int64_t seq, int per, int workers, bool solo,
                                               bool wide, int64_t t_spec, const RankTable *rtp,
                                               const int *cur_cnt, Tally *tally, double *fs,
                                               double2 *gsum, int32_t *st_id, uint8_t *st_lev) {
    const RankTable &rt = *rtp;
    const int n_act = h.n_act, split = h.split;
    const int64_t tn = h.t_next;
    const double d_spec = (double)(t_spec - tn) * kTick;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const double *__restrict__ part = A.partial;
    int nst = 0;
    for (int k0 = blockIdx.x * per; k0 < n_act; k0 += workers * per) {
        const int nt = n_act - k0 < per ? n_act - k0 : per;
        const bool valid = tid < nt;
        int id = 0, lev = 0;
        OldState old{};
        if (wide) {
            auto particle = [&]() {
                if (valid) {
                    id = rank_to_particle(A, &rt, k0 + tid);
                    old = load_old<false>(A.st, id);
                }
            };
            switch (kFinThreads / 64 / per) {
                case 1: fin_wide_sums<1>(part, k0, nt, split, gsum, fs, particle); break;
                case 2: fin_wide_sums<2>(part, k0, nt, split, gsum, fs, particle); break;
                case 4: fin_wide_sums<4>(part, k0, nt, split, gsum, fs, particle); break;
                default: fin_wide_sums<8>(part, k0, nt, split, gsum, fs, particle); break;
            }
        } else {
            // thread tid = j * per + kl: slices 4j .. 4j + 3 of target k0 + kl
            // (36 loads in flight; consecutive threads, consecutive targets:
            // coalesced), the seg partial sums then merged in order
            const int kl = tid % per, j = tid / per;
            const bool mine = kl < nt;
            const double *__restrict__ pk = part + (mine ? k0 + kl : 0);
            const int64_t cs = n_act, ss = (int64_t)9 * n_act;
            double x[36];
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int c = 0; c < 9; ++c) {
                    const int sl = 4 * j + q;
                    x[q * 9 + c] = mine && sl < split ? pk[sl * ss + c * cs] : 0.0;
                }
            if (valid) {
                id = rank_to_particle(A, &rt, k0 + tid);
                old = load_old<false>(A.st, id);
            }
            double hs[9], hc[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) hs[c] = hc[c] = 0.0;
#pragma unroll
            for (int q = 0; q < 36; ++q) two_sum_into(hs[q % 9], hc[q % 9], x[q]);
#pragma unroll
            for (int c = 0; c < 9; ++c) fs[tid * 9 + c] = hs[c] + hc[c];
            const int seg = kFinThreads / per;
            if (seg > 1) {
                __syncthreads();
                if (tid < nt) {
#pragma unroll
                    for (int c = 0; c < 9; ++c) {
                        double ts = 0.0, tc = 0.0;
                        for (int jj = 0; jj < seg; ++jj) two_sum_into(ts, tc, fs[(jj * per + tid) * 9 + c]);
                        hs[c] = ts + tc;
                    }
                }
                __syncthreads();
                if (tid < nt)
#pragma unroll
                    for (int c = 0; c < 9; ++c) fs[tid * 9 + c] = hs[c];
            }
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
            A.lvl[((seq + 1) & 1) * (int64_t)A.n + id] = (uint8_t)lev;
            // its prediction to the guessed next block time, from registers
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double xp, vp, ap;
                predict_comp(x1[c], v1[c], f[c], f[3 + c], f[6 + c], c1[c], d_spec, xp, vp, ap);
                A.pred.x[c][id] = xp;
                A.pred.v[c][id] = vp;
                A.pred.a[c][id] = ap;
            }
            st_id[nst + tid] = id;
            st_lev[nst + tid] = (uint8_t)lev;
        }
        nst += nt;
        const bool last = k0 + workers * per >= n_act;
        if (last || nst + per > kStash) {
            list_insert_stash(A, &rt, cur_cnt, solo ? tally : nullptr, st_id, st_lev, nst);
            nst = 0;
        } else {
            __syncthreads();  // fs and gsum reusable
        }
    }
    if (solo) {
        plan_next(A, h, cur_cnt, tally, dn, seq, t_spec);
        return;
    }
    if (!arrive_last(&A.scr->done_fin, (unsigned)workers)) return;
    plan_next(A, h, cur_cnt, nullptr, dn, seq, t_spec);
}

// Prediction to t_to of the particles not due in the block (all of them in
// a prediction slot), in index order (coalesced; the level lists are in no
// useful order) by workgroups wg0 .. gridDim.x - 1. A particle is due iff its
// level at the block's start (level bytes, buffer seq & 1) is L0 or more;
// the finishing workgroups predict those themselves and write their new
// levels, so each entry of the next level buffer has one writer, and no
// thread here reads a state that is being corrected.
__device__ __forceinline__ void predict_rest(const LoopArgs &A, int L0, int64_t seq, int64_t t_to,
                                             int wg0, bool all) {
    const uint8_t *__restrict__ cur = A.lvl + (seq & 1) * (int64_t)A.n;
    uint8_t *__restrict__ nxt = A.lvl + ((seq + 1) & 1) * (int64_t)A.n;
    const int stride = ((int)gridDim.x - wg0) * (int)blockDim.x;
    for (int i = ((int)blockIdx.x - wg0) * (int)blockDim.x + (int)threadIdx.x; i < A.n; i += stride) {
        const int lev = cur[i];
        if (!all && lev >= L0) continue;
        nxt[i] = (uint8_t)lev;
        predict_one(A.st, i, (double)(t_to - A.st.t[i]) * kTick, A.pred);
    }
}

// Compensated slice sums, corrector, list updates, and (last workgroup) the
// plan of the next block. Targets go in rounds of fin_per_round(split, n_act):
// with few slices seg threads per target, four slices each (the slice sums
// stored target-minor, so the loads are coalesced), merged in order; with more,
// one wave per target whose lanes are (component, group) -- 9 x 7 -- each
// summing every 7th slice of its component (stored slice-minor, loads of a
// component coalesced), the 7 group sums then merged in order through LDS.
// The corrected particles' list slots are reserved once per level for up
// to kStash particles. Every corrected particle is then predicted, from
// registers, to the guessed next block time t_spec (the step of the highest
// occupied level after t_next); the workgroups without targets (all of them,
// after their targets, when every one has some) predict the particles not
// due to t_spec as well, in index order, so no separate prediction pass runs
// before the next evaluation. The plan records whether the guess held; if
// not, the next slot is a prediction slot: its evaluation does nothing and
// its finishing kernel predicts every particle to the planned time and
// hands the same plan on.
__global__ __launch_bounds__(kFinThreads) void k_bl_finish(LoopArgs A, int64_t seq) {
    const LoopDesc *__restrict__ d = A.desc + (seq & 1);
    LoopDesc *dn = A.desc + ((seq + 1) & 1);
    const DescHead h = load_head(d);
    const int n_act = h.n_act;
    if (n_act == 0) {
        // nothing due before t_end: carry the final descriptor forward
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            *dn = *d;
            if (A.nact_log) {
                int32_t *e = A.nact_log + 2 * ((seq + 1) & A.log_mask);
                e[0] = e[1] = 0;
            }
        }
        return;
    }
    const int64_t tn = h.t_next;
    if (!h.pred_ok) {
        // prediction slot: every particle to the planned block's time (the
        // last finishing kernel's guess was wrong); the block runs next slot
        predict_rest(A, h.L0, seq, tn, 0, true);
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            *dn = *d;
            dn->pred_ok = 1;
            if (A.nact_log) {
                int32_t *e = A.nact_log + 2 * ((seq + 1) & A.log_mask);
                e[0] = n_act;
                e[1] = h.split;
            }
        }
        return;
    }
    // the guess of the next block time: the highest occupied level (always
    // active) is due again after its step, unless a correction changes it
    const int64_t t_spec = tn + ((int64_t)1 << (kTickBits - h.lv_hi));
    const int split = h.split;
    const bool wide = split > kFinSplitNarrow;
    const int per = fin_per_round(split, n_act);
    const int workers = fin_workers(n_act, split);
    if ((int)blockIdx.x >= workers) {
        // no targets: the particles not due, to t_spec
        predict_rest(A, h.L0, seq, t_spec, workers, false);
        return;
    }
    const bool solo = workers == 1;  // no other workgroup: tallies in LDS, no device atomics
    __shared__ double fs[kFinThreads * 9];
    __shared__ double2 gsum[kFinThreads];  // wide: group sums, [wave][component * 7 + group]
    __shared__ int32_t st_id[kStash];
    __shared__ uint8_t st_lev[kStash];
    __shared__ RankTable rt;
    __shared__ int cur_cnt[kLevels];
    __shared__ Tally tally;
    if (threadIdx.x < kLevels) {
        cur_cnt[threadIdx.x] = h.my_cnt;
        tally.reb[threadIdx.x] = 0u;
    }
    if (threadIdx.x == 0) tally.app = 0u;
    rank_table_from(&rt, h);  // ends with a barrier
    finish_targets(A, h, d, dn, seq, per, workers, solo, wide, t_spec, &rt, cur_cnt, &tally, fs,
                   gsum, st_id, st_lev);
    // every workgroup has targets: the particles not due afterwards
    if (workers == (int)gridDim.x) predict_rest(A, h.L0, seq, t_spec, 0, false);
}

// ---------------------------------------------------------------- set-up

__global__ void k_bl_setup_init(LoopArgs A) {
    LoopScratch *scr = A.scr;
    for (int i = threadIdx.x; i < kLevels; i += blockDim.x) scr->reb[i][0] = 0u;
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
        if (lcount[L] > 0) lbase[L] = add_agent(&A.scr->reb[L][0], lcount[L]);
    __syncthreads();
    if (good) {
        level_list(A, 0, lev)[lbase[lev] + rank] = i;
        A.lvl[i] = (uint8_t)lev;  // level buffer 0: slot 0 reads it
    }
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
        const int c = invalid ? 0 : (int)scr->reb[L][0];
        s_cnt[L] = c;
        d->cnt[L] = c;
        scr->reb[L][0] = 0u;
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
        if (A.nact_log) A.nact_log[0] = A.nact_log[1] = 0;
        return;
    }
    if (threadIdx.x == 0) scr->bad = 0u;
    if (threadIdx.x < 64) plan_block(A, d, s_cnt, (int64_t)tmax, 0ull, 0, 0, 0, -1);
}

}  // namespace

// One round of resident evaluation workgroups (one wave each): two per SIMD,
// four for the mixed form, whose evaluation kernel fits their registers.
int bl_eval_grid(h6_ctx ctx, int precision) {
    return ctx->n_cu * (precision == H6_MIXED ? 16 : 8);
}

int64_t bl_list_ints(int64_t n, int nl) { return 2 * (int64_t)nl * n + (2 * n + 3) / 4; }

hipError_t bl_setup(h6_ctx ctx, const LoopArgs &A) {
    hipLaunchKernelGGL(k_bl_setup_init, dim3(1), dim3(64), 0, ctx->stream, A);
    hipLaunchKernelGGL(k_bl_setup_scan, dim3((A.n + kScanThreads - 1) / kScanThreads),
                       dim3(kScanThreads), 0, ctx->stream, A);
    hipLaunchKernelGGL(k_bl_setup_plan, dim3(1), dim3(64), 0, ctx->stream, A);
    return hipGetLastError();
}

hipError_t bl_enqueue_block(h6_ctx ctx, const LoopArgs &A, int precision, int64_t seq) {
    // with the measurement hook on, both dispatches carry an end event (part
    // of the dispatch itself: no marker packet in the stream); a dispatch's
    // span runs from the end of the work before it (ctx->bl_mark)
    const bool prof = ctx->prof;
    hipEvent_t ev_eval = nullptr, ev_fin = nullptr;
    hipError_t pe = hipSuccess;
    if (prof && ((pe = prof_event(ctx, &ev_eval)) != hipSuccess ||
                 (pe = prof_event(ctx, &ev_fin)) != hipSuccess))
        return pe;
    auto push = [&](hipEvent_t e0, hipEvent_t e1, int kind) {
        hipError_t r = hipGetLastError();
        return r != hipSuccess ? r : prof_push_seq(ctx, e0, e1, precision, seq, kind);
    };
    const bool skip = self_pair_masked(A.eps2, precision);
    const bool mixed = precision == H6_MIXED;
#define H6_BL_EVAL(M, S)                                                                    \
    hipExtLaunchKernelGGL((k_bl_eval<M, S>), dim3(A.eval_grid), dim3(64), 0, ctx->stream, \
                          nullptr, ev_eval, 0u, A, seq)
    if (mixed) {
        if (skip) H6_BL_EVAL(true, true); else H6_BL_EVAL(true, false);
    } else {
        if (skip) H6_BL_EVAL(false, true); else H6_BL_EVAL(false, false);
    }
#undef H6_BL_EVAL
    if (prof && (pe = push(ctx->bl_mark, ev_eval, 2)) != hipSuccess) return pe;
    hipExtLaunchKernelGGL(k_bl_finish, dim3(kFinLaunch), dim3(kFinThreads), 0, ctx->stream,
                          nullptr, ev_fin, 0u, A, seq);
    if (prof) {
        if (ctx->prof_level >= 2 && (pe = push(ev_eval, ev_fin, 4)) != hipSuccess) return pe;
        ctx->bl_mark = ev_fin;
    }
    return hipGetLastError();
}

}  // namespace h6
