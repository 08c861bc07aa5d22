// C ABI of libh6: argument validation, scratch ownership, error mapping,
// and the native block-step driver loop. Kernels live in eval.hip and
// steps.hip; this file only validates, allocates and sequences.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>

#include "h6_internal.h"

using namespace h6;

// Scratch of the allocation-free evaluation (h6_evaluate_noalloc): one copy
// per GPU the library runs on, held until the process ends. Host code uses
// the per-device address from hipGetSymbolAddress, never the array's name
// (a host-side stand-in that is no device address).
static __device__ __align__(256) double scratch[H6_NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {

// Pinned host staging: [0, 16) block readback, [64, 68) flags,
// [128, 168) energy, two block-loop descriptor slots.
constexpr size_t kHostBytes = 2048;
constexpr size_t kHostSlot0 = 1024;
constexpr size_t kHostSlot1 = 1536;
static_assert(sizeof(LoopDesc) <= kHostSlot1 - kHostSlot0 && kHostSlot1 + sizeof(LoopDesc) <= kHostBytes,
              "descriptor slots");

int fail_hip(h6_ctx ctx, hipError_t e, const char *what) {
    if (ctx) {
        char buf[256];
        std::snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
        ctx->last_error = buf;
    }
    return H6_EHIP;
}

int fail_arg(h6_ctx ctx, const char *what) {
    if (ctx) ctx->last_error = what;
    return H6_EINVAL;
}

#define H6_TRY(ctx, call, what)                            \
    do {                                                   \
        hipError_t e_ = (call);                            \
        if (e_ != hipSuccess) return fail_hip(ctx, e_, what); \
    } while (0)

bool state_ok(const h6_state *st, bool need_time) {
    if (!st || !st->m) return false;
    for (int c = 0; c < 3; ++c)
        if (!st->x[c] || !st->v[c] || !st->a[c] || !st->j[c] || !st->s[c] || !st->c[c]) return false;
    if (need_time && (!st->t || !st->dt)) return false;
    return true;
}

bool pred_ok(const h6_pred *p) {
    if (!p) return false;
    for (int c = 0; c < 3; ++c)
        if (!p->x[c] || !p->v[c] || !p->a[c]) return false;
    return true;
}

bool force_ok(const h6_force *f) {
    if (!f) return false;
    for (int c = 0; c < 3; ++c)
        if (!f->a[c] || !f->j[c] || !f->s[c]) return false;
    return true;
}

bool precision_ok(int p) { return p == H6_FP64 || p == H6_MIXED || p == H6_EX || p == H6_SP; }

bool params_ok(const h6_params *p) {
    return p && std::isfinite(p->eta) && p->eta > 0.0 && p->lev_min >= 0 &&
           p->lev_max >= p->lev_min && p->lev_max <= kTickBits &&
           precision_ok(p->precision) &&
           (p->host_loop == 0 || p->host_loop == 1);
}

int check_n(h6_ctx ctx, int64_t n) {
    if (n < 1 || n > ctx->n_max) return fail_arg(ctx, "particle count out of range");
    return H6_OK;
}

SrcPtrs src_from_pred(const h6_pred *p, const double *m) {
    SrcPtrs s;
    for (int c = 0; c < 3; ++c) {
        s.x[c] = p->x[c];
        s.v[c] = p->v[c];
        s.a[c] = p->a[c];
        s.j[c] = nullptr;
    }
    s.m = m;
    return s;
}

OutPtrs out_from_force(const h6_force *f) {
    OutPtrs o;
    for (int c = 0; c < kMaxOut; ++c) o.p[c] = nullptr;
    for (int c = 0; c < 3; ++c) {
        o.p[c] = f->a[c];
        o.p[3 + c] = f->j[c];
        o.p[6 + c] = f->s[c];
    }
    return o;
}

int read_flags(h6_ctx ctx) {
    int32_t *h = (int32_t *)((char *)ctx->host + 64);
    H6_TRY(ctx, hipMemcpyAsync(h, ctx->flags, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream),
           "flag readback");
    H6_TRY(ctx, hipMemsetAsync(ctx->flags, 0, sizeof(int32_t), ctx->stream), "flag reset");
    H6_TRY(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    if (h[0] & kFlagLoop) {
        ctx->last_error = "block loop: level-list index out of range";
        return H6_ESTATE;
    }
    if (h[0] & kFlagNonFinite) return H6_ENONFINITE;
    if (h[0] & kFlagDtMin) return H6_EDTMIN;
    return H6_OK;
}

constexpr int64_t kNoAllocDoubles = (int64_t)H6_NOALLOC_SCRATCH_BYTES / (int64_t)sizeof(double);
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
double *g_noalloc_ptr[kNoAllocDevices];  // device address of scratch, per device
int g_noalloc_cu[kNoAllocDevices];       // compute units, per device

// Largest active set of h6_evaluate_noalloc: one slice of its partial sums
// (9 doubles per target) fits the scratch.
int64_t n_noalloc_max_act() { return kNoAllocDoubles / 9; }

}  // namespace

namespace h6 {

static int timing_key(h6_ctx ctx, int order, int kind, int block, int ipl, int precision,
                      int bin);

// Algorithmic HBM bytes of the measured kernels (each datum moved once):
// an order-2 evaluation reads the predicted x, v, a and the mass of every
// source (80 B), the predicted state and list entry of every target (76 B)
// and writes 9 doubles per target and slice; predicting a particle reads
// x, v, a, j, s, c and t (152 B) and writes x, v, a (72 B); the finishing
// kernel reads the slice sums (72 B per slice) and, per active particle, its
// list entry and old x, v, a, j, s and step (132 B), and writes x, v, a, j,
// s, c, t, step, a list entry (164 B) and the predicted x, v, a (72 B), and
// predicts every inactive particle (224 B each).
constexpr double kSliceBytes = 72.0;
constexpr double kPredictBytes = 224.0;
constexpr double kFinishStateBytes = 368.0;
static double eval_bytes(double n_src, double n_act, int split) {
    return 80.0 * n_src + n_act * (76.0 + kSliceBytes * (split > 1 ? split : 0));
}

// A timing event from the pool, held until the next resolve.
hipError_t prof_event(h6_ctx ctx, hipEvent_t *e) {
    if (!ctx->event_pool.empty()) {
        *e = ctx->event_pool.back();
        ctx->event_pool.pop_back();
    } else {
        // timestamps only: no system-scope cache flush at the marker
        hipError_t r = hipEventCreateWithFlags(e, hipEventDisableSystemFence);
        if (r != hipSuccess) return r;
    }
    ctx->prof_held.push_back(*e);
    return hipSuccess;
}

hipError_t prof_events(h6_ctx ctx, hipEvent_t *e0, hipEvent_t *e1) {
    hipError_t r = prof_event(ctx, e0);
    return r != hipSuccess ? r : prof_event(ctx, e1);
}

hipError_t prof_begin(h6_ctx ctx, hipEvent_t *e0, hipEvent_t *e1) {
    hipError_t r = prof_events(ctx, e0, e1);
    if (r != hipSuccess) return r;
    return hipEventRecord(*e0, ctx->stream);
}

hipError_t prof_end(h6_ctx ctx, hipEvent_t e0, hipEvent_t e1, int order, const EvalConfig &cfg,
                    int precision, int64_t n_act, double interactions) {
    hipError_t r = hipEventRecord(e1, ctx->stream);
    if (r != hipSuccess) return r;
    int bin = 0;
    for (int64_t na = n_act; na > 1; na >>= 1) ++bin;
    const int key = timing_key(ctx, order, cfg.kind, cfg.block, cfg.ipl, precision, bin);
    const double n_src = n_act > 0 ? interactions / (double)n_act : 0.0;
    const double bytes = order == 2 ? eval_bytes(n_src, (double)n_act, cfg.n_split) : 0.0;
    ctx->pending.push_back({e0, e1, key, interactions, -1, precision, 0, bytes});
    return hipSuccess;
}

// Device-loop launch (kind 2 evaluation, 4 finishing kernel): its active
// count is known only on the device; the block log ((n_act, split) per slot
// sequence number, split -1 for a prediction slot) resolves it.
hipError_t prof_push_seq(h6_ctx ctx, hipEvent_t e0, hipEvent_t e1, int precision, int64_t seq,
                         int kind) {
    ctx->pending.push_back({e0, e1, -1, 0.0, seq, precision, kind, 0.0});
    return hipSuccess;
}

static int timing_key(h6_ctx ctx, int order, int kind, int block, int ipl, int precision,
                      int bin) {
    for (size_t q = 0; q < ctx->timings.size(); ++q) {
        const h6_eval_timing &t = ctx->timings[q];
        if (t.order == order && t.kind == kind && t.block == block && t.ipl == ipl &&
            t.precision == precision && t.nact_log2 == bin)
            return (int)q;
    }
    h6_eval_timing t = {order, kind, block, ipl, precision, bin, 0, 0.0, 0.0, 0.0};
    ctx->timings.push_back(t);
    return (int)ctx->timings.size() - 1;
}

hipError_t prof_resolve(h6_ctx ctx) {
    std::vector<int32_t> log;
    for (const auto &p : ctx->pending) {
        float ms = 0.0f;
        hipError_t r = hipEventElapsedTime(&ms, p.e0, p.e1);
        if (r != hipSuccess) return r;
        int key = p.key;
        double inter = p.interactions, bytes = p.bytes;
        if (key < 0) {
            if (log.empty()) {
                log.resize(2 * ((size_t)ctx->bl_log_mask + 1));
                r = hipMemcpy(log.data(), ctx->bl_log, log.size() * sizeof(int32_t),
                              hipMemcpyDeviceToHost);
                if (r != hipSuccess) return r;
            }
            const size_t e = 2 * (size_t)(p.seq & ctx->bl_log_mask);
            const int64_t na = log[e];
            const int split = log[e + 1];
            const bool pslot = split < 0;  // prediction slot: no evaluation
            int bin = -1;  // empty block (nothing evaluated)
            for (int64_t q = na; q >= 1; q >>= 1) ++bin;
            if (pslot) bin = -2;
            key = p.kind == 2 ? timing_key(ctx, 2, 2, 64, 2, p.precision, bin)
                              : timing_key(ctx, 2, p.kind, 0, 0, p.precision, bin);
            const double n = (double)ctx->bl_n;
            inter = (double)na * n;
            if (pslot) inter = 0.0;
            if (na == 0 || (pslot && p.kind == 2))
                bytes = 0.0;
            else if (pslot)
                bytes = kPredictBytes * n;
            else if (p.kind == 2)
                bytes = eval_bytes(n, (double)na, split);
            else
                bytes = (double)na * (kFinishStateBytes + kSliceBytes * split) +
                        kPredictBytes * (n - (double)na);
        }
        h6_eval_timing &t = ctx->timings[key];
        t.launches += 1;
        t.interactions += inter;
        t.kernel_ms += ms;
        t.bytes += bytes;
    }
    ctx->pending.clear();
    // every event back to the pool but the device loop's current mark,
    // which the next evaluation's timing starts from
    for (hipEvent_t e : ctx->prof_held)
        if (e != ctx->bl_mark) ctx->event_pool.push_back(e);
    ctx->prof_held.clear();
    if (ctx->bl_mark) ctx->prof_held.push_back(ctx->bl_mark);
    return hipSuccess;
}

}  // namespace h6

extern "C" {

int h6_self_pair_masked(double eps, int precision) {
    if (!std::isfinite(eps) || eps < 0.0 || !precision_ok(precision)) return H6_EINVAL;
    return self_pair_masked(eps * eps, precision) ? 1 : 0;
}

const char *h6_strerror(int code) {
    switch (code) {
        case H6_OK: return "ok";
        case H6_EINVAL: return "invalid argument";
        case H6_ENOMEM: return "out of device memory";
        case H6_EHIP: return "HIP runtime error";
        case H6_ESTATE: return "invalid state";
        case H6_EDTMIN: return "time step below 2^-lev_max";
        case H6_ENONFINITE: return "non-finite result";
        default: return "unknown error";
    }
}

const char *h6_last_error(h6_ctx ctx) { return ctx ? ctx->last_error.c_str() : ""; }

int h6_create(h6_ctx *out, int64_t n_max, double eps, void *hip_stream) {
    if (!out) return H6_EINVAL;
    *out = nullptr;
    if (n_max < 1 || n_max > kMaxParticles || !std::isfinite(eps) || eps < 0.0) return H6_EINVAL;
    h6_ctx ctx = new (std::nothrow) h6_ctx_s;
    if (!ctx) return H6_ENOMEM;
    ctx->n_max = n_max;
    ctx->eps = eps;
    ctx->eps2 = eps * eps;
    ctx->stream = (hipStream_t)hip_stream;
    hipError_t e = hipGetDevice(&ctx->device);
    int n_cu = 0;
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device);
    if (e != hipSuccess) {
        delete ctx;
        return H6_EHIP;
    }
    ctx->n_cu = n_cu > 0 ? n_cu : 256;
    // partial sums: n_split * ncomp * n_act doubles, n_split * n_act <= cap
    const int64_t cap_pairs = std::max<int64_t>(2 * n_max, (int64_t)1 << 21);
    ctx->partial_cap = 9 * cap_pairs;
    ctx->sched_blocks = sched_blocks_for(n_max);
    const int64_t eb = energy_blocks_for(n_max);
    bool ok = hipMalloc(&ctx->partial, sizeof(double) * ctx->partial_cap) == hipSuccess &&
              hipMalloc(&ctx->sched64, sizeof(int64_t) * (2 + ctx->sched_blocks)) == hipSuccess &&
              hipMalloc(&ctx->sched32, sizeof(int32_t) * (1 + 2 * ctx->sched_blocks)) == hipSuccess &&
              hipMalloc(&ctx->counters, sizeof(unsigned) * 8) == hipSuccess &&
              hipMalloc(&ctx->flags, sizeof(int32_t) * 4) == hipSuccess &&
              hipMalloc(&ctx->ered, sizeof(double) * (8 + 10 * eb)) == hipSuccess &&
              hipMalloc(&ctx->bl_desc, 2 * sizeof(LoopDesc)) == hipSuccess &&
              hipMalloc(&ctx->bl_scr, sizeof(LoopScratch)) == hipSuccess &&
              hipEventCreateWithFlags(&ctx->bl_ev[0], hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&ctx->bl_ev[1], hipEventDisableTiming) == hipSuccess &&
              hipHostMalloc(&ctx->host, kHostBytes, hipHostMallocDefault) == hipSuccess;
    if (ok) {
        ok = hipMemset(ctx->counters, 0, sizeof(unsigned) * 8) == hipSuccess &&
             hipMemset(ctx->flags, 0, sizeof(int32_t) * 4) == hipSuccess &&
             hipDeviceSynchronize() == hipSuccess;
    }
    if (!ok) {
        (void)hipGetLastError();
        h6_destroy(ctx);
        return H6_ENOMEM;
    }
    *out = ctx;
    return H6_OK;
}

int h6_destroy(h6_ctx ctx) {
    if (!ctx) return H6_OK;
    if (ctx->partial || ctx->sched64) (void)hipStreamSynchronize(ctx->stream);
    if (ctx->partial) (void)hipFree(ctx->partial);
    if (ctx->sched64) (void)hipFree(ctx->sched64);
    if (ctx->sched32) (void)hipFree(ctx->sched32);
    if (ctx->counters) (void)hipFree(ctx->counters);
    if (ctx->flags) (void)hipFree(ctx->flags);
    if (ctx->ered) (void)hipFree(ctx->ered);
    if (ctx->host) (void)hipHostFree(ctx->host);
    if (ctx->bl_desc) (void)hipFree(ctx->bl_desc);
    if (ctx->bl_scr) (void)hipFree(ctx->bl_scr);
    if (ctx->bl_lists) (void)hipFree(ctx->bl_lists);
    if (ctx->bl_log) (void)hipFree(ctx->bl_log);
    for (hipEvent_t e : ctx->bl_ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : ctx->prof_held) (void)hipEventDestroy(e);  // the pending timings' events
    for (hipEvent_t e : ctx->event_pool) (void)hipEventDestroy(e);
    delete ctx;
    return H6_OK;
}

int h6_set_stream(h6_ctx ctx, void *hip_stream) {
    if (!ctx) return H6_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return H6_OK;
}

int h6_set_eval_config(h6_ctx ctx, int block, int ipl, int n_split, int small_max) {
    if (!ctx) return H6_EINVAL;
    if (block != 0 && block != 64 && block != 128 && block != 256)
        return fail_arg(ctx, "block must be 0, 64, 128 or 256");
    if (ipl != 0 && ipl != 1 && ipl != 2 && ipl != 4)
        return fail_arg(ctx, "ipl must be 0, 1, 2 or 4");
    if (n_split < 0) return fail_arg(ctx, "n_split must be >= 0");
    ctx->cfg_block = block;
    ctx->cfg_ipl = ipl;
    ctx->cfg_split = n_split;
    ctx->cfg_small = small_max < 0 ? -1 : small_max;
    return H6_OK;
}

int h6_predict(h6_ctx ctx, const h6_state *st, int64_t n, int64_t t_tick, const h6_pred *out) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(st, true) || !pred_ok(out)) return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    H6_TRY(ctx, launch_predict(ctx, st, (int)n, t_tick, 0.0, false, out), "predict");
    return H6_OK;
}

int h6_predict_dt(h6_ctx ctx, const h6_state *st, int64_t n, double dt, const h6_pred *out) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(st, false) || !pred_ok(out)) return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    if (!std::isfinite(dt)) return fail_arg(ctx, "dt not finite");
    H6_TRY(ctx, launch_predict(ctx, st, (int)n, 0, dt, true, out), "predict");
    return H6_OK;
}

int h6_evaluate(h6_ctx ctx, const h6_pred *src, const double *m, int64_t n, const int32_t *active,
                int64_t n_act, int precision, const h6_force *out) {
    if (!ctx) return H6_EINVAL;
    if (!pred_ok(src) || !m || !force_ok(out)) return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    if (n_act < 0 || n_act > ctx->n_max) return fail_arg(ctx, "n_act out of range");
    if (!active && n_act > n) return fail_arg(ctx, "n_act > n without an active list");
    if (!precision_ok(precision)) return fail_arg(ctx, "bad precision");
    if (n_act == 0) return H6_OK;
    H6_TRY(ctx,
           launch_eval(ctx, 2, precision, src_from_pred(src, m), (int)n, active, (int)n_act,
                       out_from_force(out), nullptr),
           "evaluate");
    return H6_OK;
}

int h6_evaluate_noalloc(void *hip_stream, double eps, const h6_pred *src, const double *m,
                        int64_t n, const int32_t *active, int64_t n_act, int precision,
                        const h6_force *out) {
    if (!pred_ok(src) || !m || !force_ok(out)) return H6_EINVAL;
    if (n < 1 || n > kMaxParticles || n_act < 0 || n_act > n_noalloc_max_act()) return H6_EINVAL;
    if (!active && n_act > n) return H6_EINVAL;
    if (!precision_ok(precision) || !std::isfinite(eps) || eps < 0.0) return H6_EINVAL;
    if (n_act == 0) return H6_OK;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return H6_EHIP;
    }
    if (dev < 0 || dev >= kNoAllocDevices) return H6_EINVAL;
    double *ptr = nullptr;
    int n_cu = 0;
    {
        // set-up once per device, with that device current
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        if (!g_noalloc_ptr[dev]) {
            void *p = nullptr;
            int cu = 0;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p ||
                hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) !=
                    hipSuccess) {
                (void)hipGetLastError();
                return H6_EHIP;
            }
            g_noalloc_ptr[dev] = (double *)p;
            g_noalloc_cu[dev] = cu > 0 ? cu : 256;
        }
        ptr = g_noalloc_ptr[dev];
        n_cu = g_noalloc_cu[dev];
    }
    // a context on the stack whose partial-sum scratch is the device array
    // (its string and vectors stay empty: nothing is allocated)
    h6_ctx_s c;
    c.n_max = n;
    c.eps = eps;
    c.eps2 = eps * eps;
    c.stream = (hipStream_t)hip_stream;
    c.device = dev;
    c.n_cu = n_cu;
    c.partial = ptr;
    c.partial_cap = kNoAllocDoubles;
    const hipError_t e = launch_eval(&c, 2, precision, src_from_pred(src, m), (int)n, active,
                                     (int)n_act, out_from_force(out), nullptr);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return H6_EHIP;
    }
    return H6_OK;
}

int h6_correct(h6_ctx ctx, h6_state *st, const int32_t *active, int64_t n_act, const h6_force *f,
               int64_t t_next, const h6_params *prm) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(st, true) || !active || !force_ok(f)) return fail_arg(ctx, "null array");
    if (!params_ok(prm)) return fail_arg(ctx, "bad step parameters");
    if (n_act < 0 || n_act > ctx->n_max) return fail_arg(ctx, "n_act out of range");
    if (t_next <= 0) return fail_arg(ctx, "t_next must be positive");
    H6_TRY(ctx, launch_correct(ctx, st, active, (int)n_act, f, t_next, 0.0, prm, false), "correct");
    return H6_OK;
}

int h6_correct_shared(h6_ctx ctx, h6_state *st, int64_t n, const h6_force *f, double dt) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(st, false) || !force_ok(f)) return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    if (!std::isfinite(dt) || dt <= 0.0) return fail_arg(ctx, "dt must be positive");
    H6_TRY(ctx, launch_correct(ctx, st, nullptr, (int)n, f, 0, dt, nullptr, true), "correct");
    return H6_OK;
}

int h6_init_forces(h6_ctx ctx, h6_state *st, int64_t n) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(st, false)) return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    // pass 1: a, j from x, v
    SrcPtrs s1;
    for (int c = 0; c < 3; ++c) {
        s1.x[c] = st->x[c];
        s1.v[c] = st->v[c];
        s1.a[c] = nullptr;
        s1.j[c] = nullptr;
    }
    s1.m = st->m;
    OutPtrs o1;
    for (int c = 0; c < kMaxOut; ++c) o1.p[c] = nullptr;
    for (int c = 0; c < 3; ++c) {
        o1.p[c] = st->a[c];
        o1.p[3 + c] = st->j[c];
    }
    H6_TRY(ctx, launch_eval(ctx, 1, H6_FP64, s1, (int)n, nullptr, (int)n, o1, nullptr), "init pass 1");
    // pass 2: s, c with the pass-1 a and j as source acceleration and jerk
    SrcPtrs s2 = s1;
    for (int c = 0; c < 3; ++c) {
        s2.a[c] = st->a[c];
        s2.j[c] = st->j[c];
    }
    OutPtrs o2;
    for (int c = 0; c < kMaxOut; ++c) o2.p[c] = nullptr;
    for (int c = 0; c < 3; ++c) {
        o2.p[6 + c] = st->s[c];
        o2.p[9 + c] = st->c[c];
    }
    H6_TRY(ctx, launch_eval(ctx, 3, H6_FP64, s2, (int)n, nullptr, (int)n, o2, nullptr), "init pass 2");
    return H6_OK;
}

int h6_initial_steps(h6_ctx ctx, h6_state *st, int64_t n, double eta_s, int lev_min, int lev_max) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(st, true)) return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    if (!std::isfinite(eta_s) || eta_s <= 0.0 || lev_min < 0 || lev_max < lev_min ||
        lev_max > kTickBits)
        return fail_arg(ctx, "bad start-up step parameters");
    H6_TRY(ctx, launch_initial_steps(ctx, st, (int)n, eta_s, lev_min, lev_max), "initial steps");
    return H6_OK;
}

int h6_next_block(h6_ctx ctx, const h6_state *st, int64_t n, int32_t *active, int64_t *t_next,
                  int64_t *n_act) {
    if (!ctx) return H6_EINVAL;
    if (!st || !st->t || !st->dt || !active || !t_next || !n_act) return fail_arg(ctx, "null pointer");
    if (int rc = check_n(ctx, n)) return rc;
    H6_TRY(ctx, launch_next_block(ctx, st, (int)n, active), "next block");
    int64_t *h64 = (int64_t *)ctx->host;
    H6_TRY(ctx,
           hipMemcpyAsync(h64, ctx->sched64, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream),
           "block readback");
    H6_TRY(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    *t_next = h64[0];
    *n_act = h64[1];
    if (!ctx->pending.empty()) H6_TRY(ctx, prof_resolve(ctx), "profile events");
    return H6_OK;
}

int h6_block_step(h6_ctx ctx, h6_state *st, int64_t n, const h6_pred *pred, const h6_force *f,
                  int32_t *active, const h6_params *prm, int64_t *t_next, int64_t *n_act) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(st, true) || !pred_ok(pred) || !force_ok(f) || !active || !t_next || !n_act)
        return fail_arg(ctx, "null pointer");
    if (!params_ok(prm)) return fail_arg(ctx, "bad step parameters");
    if (int rc = check_n(ctx, n)) return rc;
    int rc = h6_next_block(ctx, st, n, active, t_next, n_act);
    if (rc) return rc;
    if (*n_act < 1) return fail_arg(ctx, "empty block");
    H6_TRY(ctx, launch_predict(ctx, st, (int)n, *t_next, 0.0, false, pred), "predict");
    H6_TRY(ctx,
           launch_eval(ctx, 2, prm->precision, src_from_pred(pred, st->m), (int)n, active,
                       (int)*n_act, out_from_force(f), nullptr),
           "evaluate");
    H6_TRY(ctx, launch_correct(ctx, st, active, (int)*n_act, f, *t_next, 0.0, prm, false), "correct");
    return H6_OK;
}

// Host-sequenced loop: one host round trip (h6_next_block) per block.
static int run_blocks_host(h6_ctx ctx, h6_state *st, int64_t n, const h6_pred *pred,
                           const h6_force *f, int32_t *active, const h6_params *prm,
                           int64_t t_end, h6_run_stats *stats) {
    h6_run_stats s = {0, 0, 0.0, 0};
    for (;;) {
        // next_block reports the smallest due time; stop once it passes t_end
        int64_t tn = 0, na = 0;
        int rc = h6_next_block(ctx, st, n, active, &tn, &na);
        if (rc) return rc;
        if (tn > t_end) break;
        H6_TRY(ctx, launch_predict(ctx, st, (int)n, tn, 0.0, false, pred), "predict");
        H6_TRY(ctx,
               launch_eval(ctx, 2, prm->precision, src_from_pred(pred, st->m), (int)n, active,
                           (int)na, out_from_force(f), nullptr),
               "evaluate");
        H6_TRY(ctx, launch_correct(ctx, st, active, (int)na, f, tn, 0.0, prm, false), "correct");
        s.blocks += 1;
        s.particle_steps += na;
        s.interactions += (double)na * (double)n;
    }
    s.t_end = t_end;
    if (stats) *stats = s;
    return read_flags(ctx);
}

// Device-resident loop: a set-up pass builds the level lists and plans
// block 0 (one readback: a state off the block grid goes to the host loop);
// then blocks are enqueued in batches, and after enqueueing batch b the host
// waits for batch b-1 and reads its descriptor copy, so the device always
// has a batch queued. Slots enqueued after the last block due are no-ops;
// batch sizes are capped by an estimate of the slots left, so that few are.
static int run_blocks_device(h6_ctx ctx, h6_state *st, int64_t n, const h6_pred *pred,
                             const h6_force *f, int32_t *active, const h6_params *prm,
                             int64_t t_end, h6_run_stats *stats) {
    const int nl = prm->lev_max - prm->lev_min + 1;
    const int64_t need = bl_list_ints(n, nl);
    if (ctx->bl_lists_cap < need) {
        H6_TRY(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
        if (ctx->bl_lists) H6_TRY(ctx, hipFree(ctx->bl_lists), "free level lists");
        ctx->bl_lists = nullptr;
        ctx->bl_lists_cap = 0;
        if (hipMalloc(&ctx->bl_lists, sizeof(int32_t) * need) != hipSuccess) {
            (void)hipGetLastError();
            ctx->bl_lists = nullptr;
            ctx->last_error = "level lists: out of device memory";
            return H6_ENOMEM;
        }
        ctx->bl_lists_cap = need;
    }
    LoopArgs A;
    A.st = *st;
    A.n = (int)n;
    A.lev_lo = prm->lev_min;
    A.nl = nl;
    A.lists = ctx->bl_lists;
    A.lvl = (uint8_t *)(ctx->bl_lists + 2 * (int64_t)nl * n);
    A.desc = ctx->bl_desc;
    A.scr = ctx->bl_scr;
    A.partial = ctx->partial;
    A.pred = *pred;
    A.eps2 = ctx->eps2;
    const double e2 = prm->eta * prm->eta;
    A.eta6 = e2 * e2 * e2;
    A.lev_min = prm->lev_min;
    A.lev_max = prm->lev_max;
    A.t_end = t_end;
    A.eval_grid = bl_eval_grid(ctx, prm->precision);
    A.one_target_small = prm->precision == H6_MIXED ? 1 : 0;
    A.pc_pairs = (unsigned)(ctx->partial_cap / 9);
    A.flags = ctx->flags;
    A.nact_log = ctx->prof_level > 0 ? ctx->bl_log : nullptr;
    A.log_mask = ctx->bl_log_mask;
    ctx->bl_n = n;

    LoopDesc *slot[2] = {(LoopDesc *)((char *)ctx->host + kHostSlot0),
                         (LoopDesc *)((char *)ctx->host + kHostSlot1)};
    H6_TRY(ctx, bl_setup(ctx, A), "block loop set-up");
    H6_TRY(ctx,
           hipMemcpyAsync(slot[0], ctx->bl_desc, sizeof(LoopDesc), hipMemcpyDeviceToHost,
                          ctx->stream),
           "block plan readback");
    H6_TRY(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    if (slot[0]->invalid) return run_blocks_host(ctx, st, n, pred, f, active, prm, t_end, stats);
    // Slots still to come after a plan, estimated from its time and highest
    // occupied level: were that level to stay the highest, the blocks come
    // one of its steps apart until t_end; a sixteenth more for prediction
    // slots. More blocks than that (a finer level appearing) only cost a
    // host round trip before the next batch; fewer leave empty slots.
    auto est_slots = [&](const LoopDesc &p) -> int64_t {
        if (p.done || p.lv_hi < 0) return 0;
        const int64_t r = ((t_end - p.t_next) >> (kTickBits - p.lv_hi)) + 1;
        return r + r / 16 + 1;
    };
    // measurement hook: each loop dispatch carries one event, at its end; an
    // evaluation's span starts at the mark (the end of the dispatch or copy
    // before it)
    if (ctx->prof) {
        H6_TRY(ctx, prof_event(ctx, &ctx->bl_mark), "profile event");
        H6_TRY(ctx, hipEventRecord(ctx->bl_mark, ctx->stream), "event record");
    }
    int64_t seq = 0;
    int next = 0;               // readback slot of the next batch
    int last = 0;               // readback slot enqueued last (0: the set-up plan)
    bool pending = false;       // a batch is queued whose plan copy is unread
    int pend = 0;               // its readback slot
    int64_t pend_slots = 0;     // and its size
    bool done = slot[0]->done != 0;
    int64_t est = est_slots(*slot[0]);
    int batch = 4;
    while (!done) {
        int64_t room = est - (pending ? pend_slots : 0);
        if (room <= 0 && pending) {
            // the queued batch should end the run: wait for it first
            H6_TRY(ctx, hipEventSynchronize(ctx->bl_ev[pend]), "event wait");
            pending = false;
            done = slot[pend]->done != 0;
            est = est_slots(*slot[pend]);
            continue;
        }
        const int nb = (int)(room < 1 ? 1 : (room < batch ? room : batch));
        for (int b = 0; b < nb; ++b, ++seq)
            H6_TRY(ctx, bl_enqueue_block(ctx, A, prm->precision, seq), "block step");
        // plan of the block after the batch: done once nothing is due before t_end
        H6_TRY(ctx,
               hipMemcpyAsync(slot[next], ctx->bl_desc + (seq & 1), sizeof(LoopDesc),
                              hipMemcpyDeviceToHost, ctx->stream),
               "block status readback");
        H6_TRY(ctx, hipEventRecord(ctx->bl_ev[next], ctx->stream), "event record");
        if (ctx->prof) {
            H6_TRY(ctx, prof_event(ctx, &ctx->bl_mark), "profile event");
            H6_TRY(ctx, hipEventRecord(ctx->bl_mark, ctx->stream), "event record");
        }
        last = next;
        if (pending) {
            H6_TRY(ctx, hipEventSynchronize(ctx->bl_ev[pend]), "event wait");
            if (slot[pend]->done) break;  // the batch just queued finds nothing to do
            est = est_slots(*slot[pend]);
        }
        pending = true;
        pend = next;
        pend_slots = nb;
        next ^= 1;
        if (batch < 64) batch *= 2;
        if (ctx->prof && (int64_t)ctx->pending.size() > (int64_t)(ctx->bl_log_mask / 2)) {
            // resolve before the block log ring wraps
            H6_TRY(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
            H6_TRY(ctx, prof_resolve(ctx), "profile events");
        }
    }
    H6_TRY(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    ctx->bl_slots = seq;
    // the copy enqueued last (or the set-up plan when nothing was due)
    const LoopDesc &d = *slot[last];
    ctx->bl_mark = nullptr;  // returned to the pool by the next resolve
    if (!ctx->pending.empty()) H6_TRY(ctx, prof_resolve(ctx), "profile events");
    if (stats) {
        stats->blocks = d.blocks;
        stats->particle_steps = d.particle_steps;
        stats->interactions = (double)d.particle_steps * (double)n;
        stats->t_end = t_end;
    }
    return read_flags(ctx);
}

int h6_run_blocks(h6_ctx ctx, h6_state *st, int64_t n, const h6_pred *pred, const h6_force *f,
                  int32_t *active, const h6_params *prm, int64_t t_end, h6_run_stats *stats) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(st, true) || !pred_ok(pred) || !force_ok(f) || !active)
        return fail_arg(ctx, "null pointer");
    if (!params_ok(prm)) return fail_arg(ctx, "bad step parameters");
    if (int rc = check_n(ctx, n)) return rc;
    // the device loop carries the FP64 and mixed kernels only
    if (prm->host_loop || prm->precision == H6_EX || prm->precision == H6_SP)
        return run_blocks_host(ctx, st, n, pred, f, active, prm, t_end, stats);
    return run_blocks_device(ctx, st, n, pred, f, active, prm, t_end, stats);
}

int h6_shared_steps(h6_ctx ctx, h6_state *st, int64_t n, const h6_pred *pred, const h6_force *f,
                    double dt, int64_t nsteps, int precision) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(st, false) || !pred_ok(pred) || !force_ok(f)) return fail_arg(ctx, "null pointer");
    if (int rc = check_n(ctx, n)) return rc;
    if (!std::isfinite(dt) || dt <= 0.0 || nsteps < 0) return fail_arg(ctx, "bad dt or step count");
    if (!precision_ok(precision)) return fail_arg(ctx, "bad precision");
    for (int64_t k = 0; k < nsteps; ++k) {
        H6_TRY(ctx, launch_predict(ctx, st, (int)n, 0, dt, true, pred), "predict");
        H6_TRY(ctx,
               launch_eval(ctx, 2, precision, src_from_pred(pred, st->m), (int)n, nullptr, (int)n,
                           out_from_force(f), nullptr),
               "evaluate");
        H6_TRY(ctx, launch_correct(ctx, st, nullptr, (int)n, f, 0, dt, nullptr, true), "correct");
    }
    return H6_OK;
}

int h6_energy(h6_ctx ctx, const h6_state *st, int64_t n, double out[5]) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(st, false) || !out) return fail_arg(ctx, "null pointer");
    if (int rc = check_n(ctx, n)) return rc;
    H6_TRY(ctx, launch_energy(ctx, st, (int)n), "energy");
    double *h = (double *)((char *)ctx->host + 128);
    H6_TRY(ctx, hipMemcpyAsync(h, ctx->ered, 5 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream),
           "energy readback");
    H6_TRY(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    std::memcpy(out, h, 5 * sizeof(double));
    return H6_OK;
}

int h6_evaluate_vjp(h6_ctx ctx, const h6_pred *src, const double *m, int64_t n,
                    const h6_force *cot, const h6_pred *grad_src, double *grad_m) {
    if (!ctx) return H6_EINVAL;
    if (!pred_ok(src) || !m || !force_ok(cot) || !pred_ok(grad_src) || !grad_m)
        return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    const double *g[9];
    for (int c = 0; c < 3; ++c) {
        g[c] = cot->a[c];
        g[3 + c] = cot->j[c];
        g[6 + c] = cot->s[c];
    }
    OutPtrs o;
    for (int c = 0; c < kMaxOut; ++c) o.p[c] = nullptr;
    for (int c = 0; c < 3; ++c) {
        o.p[c] = grad_src->x[c];
        o.p[3 + c] = grad_src->v[c];
        o.p[6 + c] = grad_src->a[c];
    }
    o.p[9] = grad_m;
    H6_TRY(ctx, launch_eval_vjp(ctx, 2, src_from_pred(src, m), g, (int)n, o, 1u << 9),
           "evaluate vjp");
    return H6_OK;
}

int h6_correct_shared_vjp(h6_ctx ctx, h6_state *cot, int64_t n, const h6_force *cot_force,
                          double dt) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(cot, false) || !force_ok(cot_force)) return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    if (!std::isfinite(dt) || dt <= 0.0) return fail_arg(ctx, "dt must be positive");
    H6_TRY(ctx, launch_correct_shared_vjp(ctx, cot, (int)n, cot_force, dt), "correct vjp");
    return H6_OK;
}

int h6_predict_dt_vjp(h6_ctx ctx, h6_state *cot, int64_t n, const h6_pred *cot_pred, double dt) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(cot, false) || !pred_ok(cot_pred)) return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    if (!std::isfinite(dt)) return fail_arg(ctx, "dt not finite");
    H6_TRY(ctx, launch_predict_dt_vjp(ctx, cot, (int)n, cot_pred, dt), "predict vjp");
    return H6_OK;
}

int h6_evaluate_vjp_active(h6_ctx ctx, const h6_pred *src, const double *m, int64_t n,
                           const int32_t *active, int64_t n_act, const h6_force *cot,
                           const h6_pred *grad_src, double *grad_m) {
    if (!ctx) return H6_EINVAL;
    if (!pred_ok(src) || !m || !pred_ok(grad_src) || !grad_m) return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    if (n_act < 0 || n_act > n) return fail_arg(ctx, "n_act out of range");
    if (n_act == 0) return H6_OK;
    if (!active || !force_ok(cot)) return fail_arg(ctx, "null array");
    const double *g[9];
    for (int c = 0; c < 3; ++c) {
        g[c] = cot->a[c];
        g[3 + c] = cot->j[c];
        g[6 + c] = cot->s[c];
    }
    OutPtrs o;
    for (int c = 0; c < kMaxOut; ++c) o.p[c] = nullptr;
    for (int c = 0; c < 3; ++c) {
        o.p[c] = grad_src->x[c];
        o.p[3 + c] = grad_src->v[c];
        o.p[6 + c] = grad_src->a[c];
    }
    o.p[9] = grad_m;
    H6_TRY(ctx, launch_eval_vjp_active(ctx, src_from_pred(src, m), g, (int)n, active, (int)n_act, o),
           "evaluate vjp (active set)");
    return H6_OK;
}

int h6_correct_vjp(h6_ctx ctx, h6_state *cot, int64_t n, const int32_t *active, int64_t n_act,
                   const int64_t *dt_old, const h6_force *cot_force) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(cot, false) || !dt_old) return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    if (n_act < 0 || n_act > n) return fail_arg(ctx, "n_act out of range");
    if (n_act == 0) return H6_OK;
    if (!active || !force_ok(cot_force)) return fail_arg(ctx, "null array");
    H6_TRY(ctx, launch_correct_block_vjp(ctx, cot, active, (int)n_act, dt_old, cot_force),
           "correct vjp (block)");
    return H6_OK;
}

int h6_predict_vjp(h6_ctx ctx, h6_state *cot, int64_t n, const int64_t *t_old, int64_t t_tick,
                   const h6_pred *cot_pred) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(cot, false) || !t_old || !pred_ok(cot_pred)) return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    H6_TRY(ctx, launch_predict_block_vjp(ctx, cot, (int)n, t_old, t_tick, cot_pred),
           "predict vjp (block)");
    return H6_OK;
}

int h6_potential(h6_ctx ctx, const h6_state *st, int64_t n, double *phi) {
    if (!ctx) return H6_EINVAL;
    if (!st || !st->m || !st->x[0] || !st->x[1] || !st->x[2] || !phi)
        return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    H6_TRY(ctx, launch_potential(ctx, st, (int)n, phi), "potential");
    return H6_OK;
}

int h6_energy_vjp(h6_ctx ctx, const h6_state *st, int64_t n, const double *cot_e,
                  h6_state *grad) {
    if (!ctx) return H6_EINVAL;
    if (!st || !grad || !st->m || !grad->m) return fail_arg(ctx, "null array");
    for (int c = 0; c < 3; ++c)
        if (!st->x[c] || !st->v[c] || !grad->x[c] || !grad->v[c]) return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    H6_TRY(ctx, launch_energy_vjp(ctx, st, (int)n, cot_e, grad), "energy gradient");
    return H6_OK;
}

int h6_init_forces_vjp(h6_ctx ctx, const h6_state *st, int64_t n, h6_state *cot) {
    if (!ctx) return H6_EINVAL;
    if (!state_ok(st, false) || !state_ok(cot, false)) return fail_arg(ctx, "null array");
    if (int rc = check_n(ctx, n)) return rc;
    // pass 2, (s, c) from (x, v, a, j, m): cotangents (sbar, cbar); adds
    // into xbar, vbar, abar, jbar, mbar
    SrcPtrs s2;
    for (int c = 0; c < 3; ++c) {
        s2.x[c] = st->x[c];
        s2.v[c] = st->v[c];
        s2.a[c] = st->a[c];
        s2.j[c] = st->j[c];
    }
    s2.m = st->m;
    const double *g2[6];
    for (int c = 0; c < 3; ++c) {
        g2[c] = cot->s[c];
        g2[3 + c] = cot->c[c];
    }
    OutPtrs o;
    for (int c = 0; c < kMaxOut; ++c) o.p[c] = nullptr;
    for (int c = 0; c < 3; ++c) {
        o.p[c] = cot->x[c];
        o.p[3 + c] = cot->v[c];
        o.p[6 + c] = cot->a[c];
        o.p[9 + c] = cot->j[c];
    }
    o.p[12] = cot->m;
    H6_TRY(ctx, launch_eval_vjp(ctx, 3, s2, g2, (int)n, o, 0x1fffu), "init vjp pass 2");
    // pass 1, (a, j) from (x, v, m): cotangents (abar, jbar) now complete
    SrcPtrs s1 = s2;
    for (int c = 0; c < 3; ++c) {
        s1.a[c] = nullptr;
        s1.j[c] = nullptr;
    }
    const double *g1[6];
    for (int c = 0; c < 3; ++c) {
        g1[c] = cot->a[c];
        g1[3 + c] = cot->j[c];
    }
    OutPtrs o1;
    for (int c = 0; c < kMaxOut; ++c) o1.p[c] = nullptr;
    for (int c = 0; c < 3; ++c) {
        o1.p[c] = cot->x[c];
        o1.p[3 + c] = cot->v[c];
    }
    o1.p[6] = cot->m;
    H6_TRY(ctx, launch_eval_vjp(ctx, 1, s1, g1, (int)n, o1, 0x7fu), "init vjp pass 1");
    return H6_OK;
}

int h6_profile_enable(h6_ctx ctx, int on) {
    if (!ctx) return H6_EINVAL;
    if (on < 0 || on > 3) return fail_arg(ctx, "bad profile level");
    H6_TRY(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    H6_TRY(ctx, prof_resolve(ctx), "profile events");
    if (on && !ctx->bl_log) {
        const int cap = 1 << 20;
        H6_TRY(ctx, hipMalloc(&ctx->bl_log, 2 * sizeof(int32_t) * cap), "block log");
        H6_TRY(ctx, hipMemset(ctx->bl_log, 0, 2 * sizeof(int32_t) * cap), "block log");
        ctx->bl_log_mask = cap - 1;
    }
    ctx->timings.clear();
    ctx->prof = on == 1 || on == 2;
    ctx->prof_level = on;
    ctx->bl_slots = 0;
    return H6_OK;
}

int h6_profile_slots(h6_ctx ctx, int32_t *out, int max, int *count) {
    if (!ctx || !count || max < 0 || (max > 0 && !out)) return fail_arg(ctx, "bad slot log read");
    H6_TRY(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    const int64_t cap = ctx->bl_log ? (int64_t)ctx->bl_log_mask + 1 : 0;
    const int64_t n = ctx->bl_slots < cap ? ctx->bl_slots : cap;
    *count = (int)n;
    if (n == 0 || max == 0) return H6_OK;
    // the run's last n slots (slot s at ring entry s & mask)
    std::vector<int32_t> ring(2 * (size_t)cap);
    H6_TRY(ctx, hipMemcpy(ring.data(), ctx->bl_log, ring.size() * sizeof(int32_t),
                          hipMemcpyDeviceToHost),
           "slot log");
    const int64_t first = ctx->bl_slots - n;
    for (int64_t k = 0; k < n && k < max; ++k) {
        const size_t e = 2 * (size_t)((first + k) & ctx->bl_log_mask);
        out[2 * k] = ring[e];
        out[2 * k + 1] = ring[e + 1];
    }
    return H6_OK;
}

int h6_profile_read(h6_ctx ctx, h6_eval_timing *out, int max, int *count) {
    if (!ctx || !count || max < 0 || (max > 0 && !out)) return fail_arg(ctx, "bad profile read");
    H6_TRY(ctx, hipStreamSynchronize(ctx->stream), "synchronize");
    H6_TRY(ctx, prof_resolve(ctx), "profile events");
    const int nrec = (int)ctx->timings.size();
    if (nrec > max) {
        *count = nrec;
        for (int q = 0; q < max; ++q) out[q] = ctx->timings[q];
        return H6_OK;
    }
    for (int q = 0; q < nrec && q < max; ++q) out[q] = ctx->timings[q];
    *count = nrec;
    return H6_OK;
}

int h6_check_status(h6_ctx ctx) {
    if (!ctx) return H6_EINVAL;
    return read_flags(ctx);
}

}  // extern "C"
