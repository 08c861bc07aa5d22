// Internal declarations of libh6 (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "h6.h"

namespace h6 {

// Particle ranges are addressed with 32-bit indices inside kernels.
constexpr int64_t kMaxParticles = (int64_t)1 << 30;
constexpr int kTickBits = H6_TICK_BITS;

// Device status flags (bit set in ctx->flags[0]).
constexpr int kFlagDtMin = 1;
constexpr int kFlagNonFinite = 2;
constexpr int kFlagLoop = 4;  // block-loop bookkeeping out of range (internal error)

// Source (j-side) arrays of an evaluation, structure of arrays.
struct SrcPtrs {
    const double *x[3], *v[3], *a[3], *j[3];
    const double *m;
};

// Output arrays by component: component c of target k of slice s lives at
// p[c][s * slice_stride + k * kstride].
constexpr int kMaxOut = 16;
struct OutPtrs {
    double *p[kMaxOut];
    int64_t kstride = 1;
};

// Whether the evaluation must mask the self pair (by index, which costs a
// compare and two selects per pair). With a softening eps the self pair has
// r = v = a = 0 and R^2 = eps^2, so each of its terms is m eps^-3 times an
// exact zero: zero while m eps^-3 is finite in the pair arithmetic, NaN
// (inf * 0) once it overflows, and 0 * inf with eps = 0. Below the limit
// eps of self_mask_eps the pair is masked; at or above it the self term is
// finite (an exact zero) for every mass below H6_SELF_MASK_MASS_F32 (the
// FP32-range arithmetics mixed, EX, SP: eps^-3 <= 2^90) or
// H6_SELF_MASK_MASS_F64 (FP64: eps^-3 <= 2^900).
inline double self_mask_eps(int precision) {
    return precision == H6_FP64 ? H6_SELF_MASK_EPS_F64 : H6_SELF_MASK_EPS_F32;
}
inline bool self_pair_masked(double eps2, int precision) {
    const double lim = self_mask_eps(precision);
    return !(eps2 >= lim * lim);  // eps below the limit (0 included)
}

// ---- device-resident block loop (blockloop.hip)
constexpr int kLevels = kTickBits + 1;  // levels 0..40: step 2^-level
constexpr int kSmall2Max = 48;          // largest active set of the source-parallel kinds
constexpr int kExtBlock = 64;           // workgroup of the EX and SP kernels (one target per lane)

// Plan of one block, written by the plan of the block before (double
// buffered by block parity) and read by the kernels of the block.
struct LoopDesc {
    int64_t t_next;          // block time (ticks)
    int64_t blocks;          // non-empty blocks planned since the loop started
    int64_t particle_steps;  // sum of their active counts
    uint64_t sel;            // bit L: list buffer holding level L
    int32_t n_act;           // active particles; 0 = nothing to do
    int32_t done;            // 1 once t_next would pass t_end
    int32_t invalid;         // set-up found a state off the block grid
    int32_t kind;            // evaluation kind: 0 tile (two targets per lane), 2 tile (one),
                             // 1 one target per wave, 3 two
    int32_t groups;          // target groups
    int32_t split;           // source slices
    int32_t slice_len;       // sources per slice
    int32_t L0;              // lowest active level
    int32_t lv_hi;           // highest occupied level
    int32_t pred_ok;         // 1: the predicted arrays hold every particle at t_next; 0: this
                             // slot only predicts them, and the block runs in the next slot
    int32_t cnt[kLevels];    // particles per level
    int32_t off[kLevels];    // first active rank of level L (L >= L0)
};

// Counters of the loop (device, zero between blocks). Every counter that
// many workgroups update in one block has a 128-byte line of its own:
// device-scope atomics on one line serialise (about 11 ns each on this
// GPU, measured), those on distinct lines proceed in parallel.
constexpr int kLineU = 32;  // unsigned per 128-byte line
struct LoopScratch {
    unsigned done_fin;             // finishing workgroups done
    unsigned pad0[kLineU - 1];
    unsigned app;                  // particles appended to level L0 - 1
    unsigned pad1[kLineU - 1];
    unsigned reb[kLevels][kLineU]; // [L][0]: size of the rebuilt list of level L (set-up: fill)
    unsigned bad;                  // set-up: particles off the block grid
    unsigned pad2[kLineU - 1];
    unsigned long long t_max;      // set-up: latest particle time
    unsigned long long due_min;    // set-up: earliest t + dt
};

// Arguments of every loop kernel.
struct LoopArgs {
    h6_state st;
    int n;
    int lev_lo, nl;       // list levels lev_lo .. lev_lo + nl - 1
    int32_t *lists;       // [2][nl][n]
    uint8_t *lvl;         // [2][n]: every particle's level at the start of slot seq, in
                          // buffer seq & 1 (after the lists, in their allocation)
    LoopDesc *desc;       // [2]
    LoopScratch *scr;
    double *partial;      // [split][9][n_act]
    h6_pred pred;         // predicted x, v, a (tile kind)
    double eps2, eta6;
    int lev_min, lev_max;
    int64_t t_end;
    int eval_grid;        // evaluation workgroups (one wave each): two per SIMD, four mixed
    int one_target_small; // 1: the source-parallel kinds take one target per wave (mixed)
    unsigned pc_pairs;    // partial capacity / 9: bound on split * n_act
    int32_t *flags;
    int32_t *nact_log;    // (n_act, split) by block sequence number (ring of pairs; split -1:
                          // a prediction slot), or NULL
    int log_mask;
};

struct EvalConfig {
    int kind;    // 0: LDS-tiled target-parallel kernel; 1: source-parallel small-set kernel
    int block;   // threads per workgroup
    int ipl;     // targets per thread (kind 0) or per wave (kind 1)
    int n_split; // source slices
};

}  // namespace h6

struct h6_ctx_s {
    int64_t n_max = 0;
    double eps = 0.0, eps2 = 0.0;
    hipStream_t stream = nullptr;
    int device = 0;
    int n_cu = 256;  // compute units of the device
    int cfg_block = 0, cfg_ipl = 0, cfg_split = 0;  // 0: automatic
    int cfg_small = -1;                             // < 0: built-in threshold
    // scratch (device)
    double *partial = nullptr;     // [n_split][ncomp][ld] partial sums
    int64_t partial_cap = 0;       // doubles
    int64_t *sched64 = nullptr;    // block minima, t_next
    int32_t *sched32 = nullptr;    // block counts, offsets, n_act
    unsigned *counters = nullptr;  // last-workgroup counters
    int32_t *flags = nullptr;      // status bits
    double *ered = nullptr;        // energy partials
    int64_t sched_blocks = 0;      // capacity of the scheduler arrays
    // pinned host staging for scheduler/energy readback
    void *host = nullptr;
    std::string last_error;
    // device-resident block loop
    h6::LoopDesc *bl_desc = nullptr;     // device, [2]
    h6::LoopScratch *bl_scr = nullptr;   // device
    int32_t *bl_lists = nullptr;         // device level lists
    int64_t bl_lists_cap = 0;            // ints
    int32_t *bl_log = nullptr;     // (n_act, split) per block sequence number (ring), profiling only
    int bl_log_mask = 0;
    hipEvent_t bl_ev[2] = {nullptr, nullptr};
    int64_t bl_n = 0;              // particle count of the current loop (profiling)
    // measurement hook (h6_profile_enable)
    struct PendingTiming {
        hipEvent_t e0, e1;
        int key;             // timing record, or -1: resolve through the block log
        double interactions;
        int64_t seq;         // block sequence number (device loop)
        int precision;
        int kind;            // device loop: 2 evaluation, 3 predictor, 4 finishing kernel
        double bytes;        // algorithmic bytes (host-shaped evaluations)
    };
    bool prof = false;   // event timing on (levels 1, 2)
    int prof_level = 0;  // 1: evaluation kernels; 2: also the device loop's other kernels;
                         // 3: no events, the device loop's slot log only
    int64_t bl_slots = 0;  // slots the last device-loop run enqueued (slot log)
    std::vector<hipEvent_t> event_pool;
    std::vector<hipEvent_t> prof_held;  // events of the pending timings (back to the pool on resolve)
    hipEvent_t bl_mark = nullptr;  // device loop: the end of the stream's work before the next
                                   // evaluation (held across resolves)
    std::vector<PendingTiming> pending;
    std::vector<h6_eval_timing> timings;
};

namespace h6 {

// Launchers: enqueue on ctx->stream, return hipError_t.
hipError_t launch_eval(h6_ctx ctx, int order, int precision, const SrcPtrs &src, int n,
                       const int32_t *active, int n_act, const OutPtrs &out,
                       EvalConfig *used);
EvalConfig choose_eval_config(h6_ctx ctx, int order, int precision, int n, int n_act);
// Compensated sum over n_split slices of ncomp partial arrays of n_act
// targets (ctx->partial, [slice][comp][target]) into out.p[out0 + comp];
// bit c of acc_mask adds to the existing value instead of overwriting.
hipError_t launch_reduce(h6_ctx ctx, int n_split, int ncomp, int out0, int n_act,
                         const OutPtrs &out, unsigned acc_mask);
int balanced_split(h6_ctx ctx, int waves_per_simd, int block, int n, int blocks_i);
// Mixed-precision order-2 kernels (eval_mixed.hip), launched with the shape
// chosen for the FP64 kernels.
hipError_t dispatch_mixed(const EvalConfig &cfg, bool skipself, dim3 grid, hipStream_t st,
                          const SrcPtrs &src, const int32_t *active, int n, int n_act, double eps2,
                          int slice_len, const OutPtrs &out, int64_t slice_stride);
// Double-single (H6_EX) and single-precision (H6_SP) order-2 kernels
// (eval_ex.hip): kExtBlock threads, one target per lane.
hipError_t dispatch_ext(int precision, bool skipself, dim3 grid, hipStream_t st, const SrcPtrs &src,
                        const int32_t *active, int n, int n_act, double eps2, int slice_len,
                        const OutPtrs &out, int64_t slice_stride);

hipError_t launch_predict(h6_ctx ctx, const h6_state *st, int n, int64_t t_tick, double dt,
                          bool shared, const h6_pred *out);
hipError_t launch_correct(h6_ctx ctx, h6_state *st, const int32_t *active, int n_act,
                          const h6_force *f, int64_t t_next, double dt, const h6_params *prm,
                          bool shared);
hipError_t launch_initial_steps(h6_ctx ctx, h6_state *st, int n, double eta_s, int lev_min,
                                int lev_max);
hipError_t launch_next_block(h6_ctx ctx, const h6_state *st, int n, int32_t *active);
hipError_t launch_energy(h6_ctx ctx, const h6_state *st, int n);

// Adjoint kernels (adjoint.hip).
hipError_t launch_eval_vjp(h6_ctx ctx, int order, const SrcPtrs &src, const double *const *cot,
                           int n, const OutPtrs &out, unsigned acc_mask);
hipError_t launch_correct_shared_vjp(h6_ctx ctx, h6_state *cot, int n, const h6_force *cf,
                                     double dt);
hipError_t launch_predict_dt_vjp(h6_ctx ctx, h6_state *cot, int n, const h6_pred *cp, double dt);
// Block-step adjoint: evaluation VJP over an active set (cot by rank, out
// dense: xbar, vbar, abar, mbar added), corrector and predictor transposes
// with per-particle steps and intervals; per-particle potential.
hipError_t launch_eval_vjp_active(h6_ctx ctx, const SrcPtrs &src, const double *const *cot, int n,
                                  const int32_t *active, int n_act, const OutPtrs &out);
hipError_t launch_correct_block_vjp(h6_ctx ctx, h6_state *cot, const int32_t *active, int n_act,
                                    const int64_t *dt_old, const h6_force *cf);
hipError_t launch_predict_block_vjp(h6_ctx ctx, h6_state *cot, int n, const int64_t *t_old,
                                    int64_t t_tick, const h6_pred *cp);
hipError_t launch_potential(h6_ctx ctx, const h6_state *st, int n, double *phi);
// Energy gradient (x, v, m of out), scaled by the device cotangent cot (NULL: 1).
hipError_t launch_energy_vjp(h6_ctx ctx, const h6_state *st, int n, const double *cot,
                             h6_state *out);

int sched_blocks_for(int64_t n);
// Measurement hook helpers (api.hip). prof_begin / prof_end bracket a
// launch with recorded events; prof_events hands out an event pair for a
// launch that records them itself (hipExtLaunchKernel), prof_push_seq
// queues such a pair for a device-loop block.
hipError_t prof_events(h6_ctx ctx, hipEvent_t *e0, hipEvent_t *e1);
hipError_t prof_event(h6_ctx ctx, hipEvent_t *e);
hipError_t prof_begin(h6_ctx ctx, hipEvent_t *e0, hipEvent_t *e1);
hipError_t prof_end(h6_ctx ctx, hipEvent_t e0, hipEvent_t e1, int order, const EvalConfig &cfg,
                    int precision, int64_t n_act, double interactions);
hipError_t prof_push_seq(h6_ctx ctx, hipEvent_t e0, hipEvent_t e1, int precision, int64_t seq,
                         int kind);
hipError_t prof_resolve(h6_ctx ctx);  // stream must be idle

// Device-resident block loop (blockloop.hip).
int bl_eval_grid(h6_ctx ctx, int precision);
int64_t bl_list_ints(int64_t n, int nl);  // list and level-byte storage, n particles, nl levels
hipError_t bl_setup(h6_ctx ctx, const LoopArgs &A);  // lists and the plan of block 0
hipError_t bl_enqueue_block(h6_ctx ctx, const LoopArgs &A, int precision, int64_t seq);
int energy_blocks_for(int64_t n);

}  // namespace h6
