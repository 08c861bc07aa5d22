/*
 * h6.h -- C ABI of libh6, a 6th-order Hermite direct N-body library for one
 * AMD Instinct MI355X (gfx950).
 *
 * The calls follow the paper's statement of the method (Goz et al.,
 * "Direct N-body code on low-power embedded ARM GPUs"):
 *   - Sec. 3, the three stages of the 6th-order Hermite scheme: predict
 *     (h6_predict), evaluate acceleration, jerk and snap (h6_evaluate),
 *     correct (h6_correct);
 *   - Sec. 3 item 3: the time step (generalized Aarseth criterion, inside
 *     h6_correct / h6_initial_steps), energy and angular momentum
 *     (h6_energy) computed on the device;
 *   - Sec. 3 item 4 (kernel steps i-iv): the evaluation stages source
 *     particles through on-chip local memory and skips the self term;
 *   - Sec. 3 item 6: the evaluation arithmetic is selectable (H6_FP64,
 *     H6_MIXED, and the paper's extended H6_EX and single H6_SP);
 *   - Sec. 2: block time stepping (h6_next_block and the power-of-two
 *     step rule in h6_correct; h6_run_blocks runs the whole loop);
 *   - reverse mode of the shared- and block-step paths (the *_vjp calls)
 *     and the per-particle potential (h6_potential) for energy losses.
 *
 * Conventions shared by every call:
 *   - Particle data lives in caller-owned DEVICE memory as structure of
 *     arrays: one contiguous double array per vector component. The
 *     library never frees caller memory. A context owns only its scratch
 *     (partial sums, scheduler and reduction buffers), sized at creation.
 *   - Times and steps are int64 counts of ticks of 2^-H6_TICK_BITS time
 *     units; block steps are powers of two, level L meaning 2^-L.
 *   - Every call enqueues work on the context's HIP stream and returns
 *     without waiting, except those marked "synchronizes".
 *   - Errors are negative return codes; nothing aborts or throws. Arguments
 *     are validated before any HIP call. A HIP failure returns H6_EHIP
 *     and its text is kept for h6_last_error. A context is not
 *     thread-safe; distinct contexts are independent.
 *   - Softening is Plummer: the pair potential is -m / sqrt(r^2 + eps^2).
 *     With eps > 0 the self term is exactly zero; with eps == 0 it is
 *     skipped explicitly (particles must then never coincide). The
 *     FP32-based arithmetics skip it too when eps^2 is below the smallest
 *     normal FP32 number (eps below about 1.1e-19), where it rounds away.
 */
#ifndef H6_H
#define H6_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define H6_TICK_BITS 40

/* Return codes. */
enum {
    H6_OK = 0,
    H6_EINVAL = -1,     /* bad argument: null pointer, size out of range */
    H6_ENOMEM = -2,     /* device scratch allocation failed */
    H6_EHIP = -3,       /* a HIP runtime call failed; see h6_last_error */
    H6_ESTATE = -4,     /* call not valid in the context's current state */
    H6_EDTMIN = -5,     /* a step fell below 2^-lev_max (step clamped) */
    H6_ENONFINITE = -6  /* a corrected quantity was not finite */
};

/* Evaluation arithmetic (Sec. 3 item 6: double, an extended type of about
 * 48 significand bits with single-precision exponents, or single). The
 * predictor, corrector and step rule are FP64 in every case. */
enum {
    H6_FP64 = 0,  /* all pair arithmetic and sums in IEEE double */
    H6_MIXED = 1, /* double position and velocity differences and accumulators,
                     float pair math */
    H6_EX = 2,    /* double-single ("float-float") pair arithmetic and
                     per-slice sums, float operations only */
    H6_SP = 3     /* single-precision pair arithmetic and per-slice sums */
};

typedef struct h6_ctx_s *h6_ctx;

/* Integrator state: device arrays of length n (caller-owned). */
typedef struct {
    double *x[3], *v[3];        /* position, velocity at time t */
    double *a[3], *j[3], *s[3]; /* acceleration, jerk, snap at t */
    double *c[3];               /* crackle at t (start-up or interpolated) */
    double *m;                  /* masses */
    int64_t *t;                 /* particle time, ticks */
    int64_t *dt;                /* particle step, ticks (power of two) */
} h6_state;

/* Predicted sources: device arrays of length n (caller-owned). */
typedef struct {
    double *x[3], *v[3], *a[3];
} h6_pred;

/* Evaluated acceleration, jerk, snap: device arrays of length n_act. */
typedef struct {
    double *a[3], *j[3], *s[3];
} h6_force;

/* Block-step parameters. */
typedef struct {
    double eta;    /* accuracy parameter of the 6th-order criterion */
    int lev_min;   /* largest step 2^-lev_min */
    int lev_max;   /* smallest step 2^-lev_max (below: H6_EDTMIN) */
    int precision; /* H6_FP64, H6_MIXED, H6_EX or H6_SP for the evaluation;
                      H6_EX and H6_SP always run the host loop */
    int host_loop; /* h6_run_blocks: 0 device-resident loop, 1 one host
                      round trip per block (h6_block_step repeated) */
} h6_params;

/* Counters filled by h6_run_blocks. */
typedef struct {
    int64_t blocks;       /* block steps taken */
    int64_t particle_steps; /* sum of active counts */
    double interactions;  /* sum over blocks of n_act * n (self pair counted) */
    int64_t t_end;        /* time reached, ticks */
} h6_run_stats;

/*
 * Create a context for systems of up to n_max particles with softening
 * length eps (>= 0). hip_stream is a hipStream_t (NULL: the null stream).
 * Allocates the scratch buffers on the current device.
 * Errors: H6_EINVAL (n_max < 1 or above 2^30, eps < 0 or not finite,
 * ctx NULL),
 * H6_ENOMEM, H6_EHIP.
 */
int h6_create(h6_ctx *ctx, int64_t n_max, double eps, void *hip_stream);

/* Free the context's scratch and the context. NULL is accepted. */
int h6_destroy(h6_ctx ctx);

/* Change the stream later calls enqueue on. */
int h6_set_stream(h6_ctx ctx, void *hip_stream);

/*
 * Launch shape of h6_evaluate. Active sets of at most small_max targets go
 * to a source-parallel kernel (lanes over sources, no LDS) with ipl targets
 * per wave (1, 2 or 4); larger ones to the LDS-tiled target-parallel kernel
 * with the given threads per workgroup (64, 128 or 256) and targets per
 * thread (1 or 2; 4 counts as 2 there). n_split: number of source slices
 * the sum is split into (>= 1). 0 keeps the built-in choice for block, ipl
 * and n_split; small_max < 0 keeps the built-in threshold and 0 disables
 * the small-set kernel. Results agree to rounding for every shape. The
 * device-resident block loop chooses its own shapes. Errors: H6_EINVAL.
 */
int h6_set_eval_config(h6_ctx ctx, int block, int ipl, int n_split,
                       int small_max);

/*
 * Predictor (Sec. 3, first stage): Taylor prediction of all n particles to
 * time t_tick, each over its own interval t_tick - t[i]: position to 5th
 * order, velocity to 4th, acceleration to 3rd, from the stored a, j, s, c.
 * h6_predict_dt predicts every particle over the same interval dt (shared
 * steps; the state's t is not read).
 * Errors: H6_EINVAL (null pointer, n < 1 or n > n_max).
 */
int h6_predict(h6_ctx ctx, const h6_state *st, int64_t n, int64_t t_tick,
               const h6_pred *out);
int h6_predict_dt(h6_ctx ctx, const h6_state *st, int64_t n, double dt,
                  const h6_pred *out);

/*
 * Evaluation (Sec. 3, second stage, and kernel steps i-iv): for each target
 * k < n_act, particle i = active[k] (active may be NULL: i = k), the sums
 * over every source j != i of the softened acceleration, jerk and snap
 * from the predicted x, v, a and masses m of all n particles. Results go to
 * out at index k. precision is H6_FP64, H6_MIXED, H6_EX or H6_SP (see the
 * enum above; EX and SP accumulate per source slice in their own arithmetic,
 * and the slices are combined in FP64). n_act == 0 is a no-op.
 * Errors: H6_EINVAL (null pointer, n < 1, n > n_max, n_act < 0 or
 * n_act > n_max, n_act > n with active NULL, bad precision). Active
 * indices must lie in [0, n); they are not checked on the device.
 */
int h6_evaluate(h6_ctx ctx, const h6_pred *src, const double *m, int64_t n,
                const int32_t *active, int64_t n_act, int precision,
                const h6_force *out);

/*
 * h6_evaluate for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same evaluation and arguments as h6_evaluate (and the same kernels),
 * without a context: the softening eps and the stream (hipStream_t, NULL:
 * the null stream) are passed in. The slice partial sums go to a fixed
 * device scratch of H6_NOALLOC_SCRATCH_BYTES per GPU (32 MiB, held by
 * every GPU the library runs on until the process ends); the call
 * allocates nothing. Every call on a GPU shares that GPU's scratch, so
 * calls that overlap on one GPU (other streams, other host threads) race:
 * order them. n_act must not exceed H6_NOALLOC_SCRATCH_BYTES / 72 (466033;
 * one slice of partial sums per target). The first call on a device looks
 * up the scratch's address. Returns codes only (no context for
 * h6_last_error). Errors: H6_EINVAL (null pointer, n < 1, n_act < 0 or
 * above the limit, n_act > n with active NULL, bad precision, eps < 0 or
 * not finite), H6_EHIP.
 */
#define H6_NOALLOC_SCRATCH_BYTES (32 << 20)
int h6_evaluate_noalloc(void *hip_stream, double eps, const h6_pred *src,
                        const double *m, int64_t n, const int32_t *active,
                        int64_t n_act, int precision, const h6_force *out);

/*
 * Corrector (Sec. 3, third stage) for a block: each active particle
 * i = active[k] is due at t_next = t[i] + dt[i]. Its x, v are corrected
 * to 6th order from a, j, s at both ends of the step (old ones in st,
 * new ones in f[k]); crackle, pop and the 5th derivative at t_next come
 * from the quintic interpolant; the new step is the largest power of two
 * not above the generalized Aarseth criterion
 *   eta [(|a||s| + |j|^2) / (|c||a5| + |p|^2)]^(1/6),
 * at least lev_min, shrinking freely but growing by one level only when
 * t_next is a multiple of twice the old step. a, j, s, c, t, dt are
 * updated. Steps below 2^-lev_max and non-finite results raise flags read
 * by h6_check_status.
 * Errors: H6_EINVAL.
 */
int h6_correct(h6_ctx ctx, h6_state *st, const int32_t *active,
               int64_t n_act, const h6_force *f, int64_t t_next,
               const h6_params *prm);

/* Shared-step corrector: all n particles over the same step dt; t and dt
 * of the state are left untouched. Errors: H6_EINVAL. */
int h6_correct_shared(h6_ctx ctx, h6_state *st, int64_t n,
                      const h6_force *f, double dt);

/*
 * Start-up at t = 0, where no snap or crackle exist yet: pass 1 evaluates
 * a and j from x, v; pass 2 evaluates s and the pairwise crackle c with
 * the pass-1 a and j of every source. Writes a, j, s, c of the state.
 * Errors: H6_EINVAL.
 */
int h6_init_forces(h6_ctx ctx, h6_state *st, int64_t n);

/*
 * Initial steps: t = 0 and dt = the largest power of two not above the
 * start-up (4th-order) criterion eta_s [(|a||s|+|j|^2)/(|j||c|+|s|^2)]^(1/2),
 * between 2^-lev_max and 2^-lev_min. Errors: H6_EINVAL.
 */
int h6_initial_steps(h6_ctx ctx, h6_state *st, int64_t n, double eta_s,
                     int lev_min, int lev_max);

/*
 * Block scheduler (synchronizes): t_next = min_i (t[i] + dt[i]) and the
 * particles due at t_next, written to active (device, length >= n) in
 * increasing index order; *t_next and *n_act are host outputs.
 * Errors: H6_EINVAL, H6_EHIP.
 */
int h6_next_block(h6_ctx ctx, const h6_state *st, int64_t n,
                  int32_t *active, int64_t *t_next, int64_t *n_act);

/*
 * One whole block step (synchronizes): h6_next_block, h6_predict of all
 * particles, h6_evaluate of the active ones, h6_correct. pred (length n)
 * and f, active (length >= n) are caller-owned work arrays.
 * Errors: as the calls it makes. A step clamped at 2^-lev_max or a
 * non-finite result raises a device flag that h6_check_status reports
 * (H6_EDTMIN, H6_ENONFINITE); the step is taken either way.
 */
int h6_block_step(h6_ctx ctx, h6_state *st, int64_t n, const h6_pred *pred,
                  const h6_force *f, int32_t *active, const h6_params *prm,
                  int64_t *t_next, int64_t *n_act);

/*
 * Block steps (Sec. 2 block time steps) until every particle reaches t_end
 * (ticks, a multiple of 2^-lev_min). stats may be NULL. Synchronizes at the
 * end.
 *
 * prm->host_loop == 1: h6_block_step repeated (one host round trip per
 * block).
 *
 * prm->host_loop == 0: device-resident loop. The particles are kept in
 * per-level lists on the device; each block's plan (time, active levels
 * and count, evaluation shape) is made on the device by the block before,
 * so the host only enqueues blocks in batches and waits once per batch.
 * This needs every particle on the block grid -- its step a power of two
 * between 2^-lev_max and 2^-lev_min and its time a multiple of its step,
 * no later than any particle's time plus step -- which holds after
 * h6_initial_steps and after any block steps with the same levels; a state
 * that is not on the grid is run with the host loop instead (same results).
 * The lists take 8 * (lev_max - lev_min + 1) * n bytes of device memory
 * (and 2 n bytes of per-particle levels),
 * allocated by the first call that needs them and kept by the context
 * (H6_ENOMEM if that fails). pred and f are used as work arrays; the
 * device loop writes no forces to f. On return pred holds, from the device
 * loop, every particle predicted to the last block's time plus the step of
 * its highest occupied level (the loop predicts each next block while
 * finishing the one before); from the host loop, the last block's own
 * predicted arrays.
 *
 * Both loops take the same block sequence; the evaluation shapes (and
 * hence last-bit rounding) may differ. Errors: as h6_block_step; H6_ESTATE
 * if the device loop's list bookkeeping ever went out of range (an
 * internal error, reported instead of acted on).
 */
int h6_run_blocks(h6_ctx ctx, h6_state *st, int64_t n, const h6_pred *pred,
                  const h6_force *f, int32_t *active, const h6_params *prm,
                  int64_t t_end, h6_run_stats *stats);

/* nsteps shared steps of length dt over all n particles (asynchronous). */
int h6_shared_steps(h6_ctx ctx, h6_state *st, int64_t n, const h6_pred *pred,
                    const h6_force *f, double dt, int64_t nsteps,
                    int precision);

/*
 * Energy and angular momentum (synchronizes; Sec. 3 item 3 and Eq. (1)):
 * out[0] kinetic energy, out[1] potential energy
 * -sum_{i<j} m_i m_j / sqrt(r_ij^2 + eps^2), out[2..4] angular momentum
 * sum m x cross v. Only meaningful when all particles share one time.
 * Errors: H6_EINVAL, H6_EHIP.
 */
int h6_energy(h6_ctx ctx, const h6_state *st, int64_t n, double out[5]);

/*
 * Device status flags raised since the last call (synchronizes), then
 * cleared: H6_OK, H6_EDTMIN or H6_ENONFINITE.
 */
int h6_check_status(h6_ctx ctx);

/*
 * ---- Adjoint (reverse mode) of the shared-step path ----
 * Cotangent arrays use the same structures as the forward values. For a
 * loss L, "cotangent of y" means dL/dy. These calls give gradients of a
 * loss on the final state with respect to the initial x, v and masses,
 * through the start-up passes and unrolled shared steps (the caller keeps
 * checkpoints and replays steps forward as needed).
 */

/*
 * VJP of h6_evaluate over all n targets (active = all): from the predicted
 * sources src, masses m and the cotangents cot (length n) of the evaluated
 * a, j, s, writes the cotangents of the predicted x, v, a to grad_src
 * (overwritten) and ADDS the cotangent of the masses to grad_m. The sum is
 * the hand reversal of the pair terms, gathered over the same pairs as the
 * forward sum (no atomics). Errors: H6_EINVAL.
 */
int h6_evaluate_vjp(h6_ctx ctx, const h6_pred *src, const double *m, int64_t n,
                    const h6_force *cot, const h6_pred *grad_src,
                    double *grad_m);

/*
 * Transpose of h6_correct_shared over step dt. On entry cot holds the
 * cotangents of the corrected state (x, v, a, j, s, c); on return it holds
 * those of the state before the step (x, v, a, j, s; c set to 0, the old
 * crackle entering only the predictor), and cot_force those of the
 * evaluated a, j, s. cot->m, t, dt are not used. Errors: H6_EINVAL.
 */
int h6_correct_shared_vjp(h6_ctx ctx, h6_state *cot, int64_t n,
                          const h6_force *cot_force, double dt);

/*
 * Transpose of h6_predict_dt over interval dt: ADDS to the state cotangents
 * (x, v, a, j, s, c) the contribution of the cotangents cot_pred of the
 * predicted x, v, a. Errors: H6_EINVAL.
 */
int h6_predict_dt_vjp(h6_ctx ctx, h6_state *cot, int64_t n,
                      const h6_pred *cot_pred, double dt);

/*
 * VJP of h6_init_forces at the state st (x, v, m and the a, j it produced).
 * On entry cot holds the cotangents of a, j, s, c at t = 0; the call ADDS
 * the resulting cotangents of x, v and the masses (cot->m) into cot, and
 * uses cot->a, cot->j as work space (their pass-2 contributions are added
 * before pass 1 is reversed). Errors: H6_EINVAL.
 */
int h6_init_forces_vjp(h6_ctx ctx, const h6_state *st, int64_t n,
                       h6_state *cot);

/*
 * ---- Adjoint of the block-step path (levels frozen) ----
 * The step of every particle is treated as a constant: gradients flow
 * through the predictor, evaluation and corrector of each block along the
 * block sequence the forward run took, not through the choice of steps.
 */

/*
 * VJP of h6_evaluate over an active set (the evaluation of one block): the
 * targets are the n_act particles active[0..n_act), cot holds the
 * cotangents of their evaluated a, j, s by rank (length n_act), and the
 * sources are all n particles (predicted src, masses m). ADDS the
 * cotangents of the predicted x, v, a of every particle to grad_src and of
 * the masses to grad_m (both length n). Work: about 2 n_act n pairs (each
 * pair's source part over the active sources for every particle, then its
 * target part over all sources for the active ones); self pairs skipped.
 * Active entries must be distinct and in [0, n) (not checked on the
 * device). n_act == 0 is a no-op. Errors: H6_EINVAL.
 */
int h6_evaluate_vjp_active(h6_ctx ctx, const h6_pred *src, const double *m, int64_t n,
                           const int32_t *active, int64_t n_act, const h6_force *cot,
                           const h6_pred *grad_src, double *grad_m);

/*
 * Transpose of the block-step corrector (h6_correct) for the particles
 * active[0..n_act), each over its own step dt_old[i] (ticks, the steps held
 * before the block; length n). On entry cot holds the cotangents of the
 * corrected state; on return, for the active particles, those of the state
 * before the block (x, v, a, j, s; c set to 0, the old crackle entering
 * only the predictor), and cot_force (by rank, length n_act) those of the
 * evaluated a, j, s. Other particles' cotangents are left unchanged.
 * cot->m, t, dt are not used. Errors: H6_EINVAL.
 */
int h6_correct_vjp(h6_ctx ctx, h6_state *cot, int64_t n, const int32_t *active,
                   int64_t n_act, const int64_t *dt_old, const h6_force *cot_force);

/*
 * Transpose of h6_predict to time t_tick: ADDS to the state cotangents
 * (x, v, a, j, s, c) the contribution of the cotangents cot_pred of the
 * predicted x, v, a, each particle over its own interval t_tick - t_old[i]
 * (ticks; t_old the particle times before the block, length n).
 * Errors: H6_EINVAL.
 */
int h6_predict_vjp(h6_ctx ctx, h6_state *cot, int64_t n, const int64_t *t_old,
                   int64_t t_tick, const h6_pred *cot_pred);

/*
 * Potential of every particle (Sec. 3 item 3 diagnostics, per particle):
 * phi[i] = -sum_{j != i} m_j / sqrt(|x_j - x_i|^2 + eps^2), from st->x and
 * st->m (other fields unused). The total potential energy is
 * sum_i m_i phi[i] / 2, and the derivative of the total energy with respect
 * to m_i is |v_i|^2 / 2 + phi[i]. Errors: H6_EINVAL.
 */
int h6_potential(h6_ctx ctx, const h6_state *st, int64_t n, double *phi);

/*
 * Gradient of the total energy (Eq. (1)'s E, as h6_energy computes it:
 * E = sum_i m_i |v_i|^2 / 2 - sum_{i<j} m_i m_j / sqrt(r_ij^2 + eps^2))
 * with respect to positions, velocities and masses, for energy losses:
 * grad->x[c][i] = -g m_i a_i[c] (a the softened acceleration),
 * grad->v[c][i] = g m_i v_i[c], grad->m[i] = g (|v_i|^2 / 2 + phi_i) with
 * phi_i the potential of h6_potential. g is the cotangent of E: cot_e
 * points to one double in device memory (so that a loss's gradient needs
 * no host round trip), or is NULL for g = 1. Reads st->x, st->v, st->m;
 * overwrites grad->x, grad->v, grad->m (other fields unused). O(n^2) pair
 * work. Errors: H6_EINVAL.
 */
int h6_energy_vjp(h6_ctx ctx, const h6_state *st, int64_t n, const double *cot_e,
                  h6_state *grad);

/*
 * Measurement hook: while enabled (on = 1), HIP events bracket every a/j/s
 * evaluation kernel the context launches (on its stream), and the event
 * durations are accumulated per kernel instantiation and per power-of-two
 * bin of the active-set size. In the device-resident loop both dispatches
 * of a slot carry one event each, at their end (part of the dispatch: no
 * marker packet in the stream), and a dispatch is timed from the end of
 * the work before it on the stream (the other kernel, the loop's start or
 * a plan readback), launch latency included. on = 2 also reports the
 * loop's finishing kernel of every block (records of kind 4, binned by the
 * block's active count like its evaluation). on = 3 records no events (nothing is
 * added to the dispatches, for an external tracer) and keeps only the
 * device-resident loop's slot log. on = 0 turns the hook off. Enabling
 * clears the records. h6_profile_read (synchronizes) copies up to max
 * records to out and sets *count.
 * Errors: H6_EINVAL (on outside 0..3), H6_EHIP.
 *
 * h6_profile_slots (synchronizes): the slot log of the last device-loop
 * h6_run_blocks call made with the hook on (any level): for each slot it
 * enqueued, in launch order, one evaluation and one finishing dispatch, the
 * pair (n_act, split) -- the slot's active count and source slices; split
 * -1 marks a prediction slot (its evaluation does nothing, its finishing
 * kernel predicts every particle to the planned block time), n_act 0 a
 * slot after the last due block. Copies up to max pairs (2 max int32) to
 * out and sets *count to the number of slots logged (the last 2^20 of the
 * run). Errors: H6_EINVAL, H6_EHIP.
 */
typedef struct {
    int order;      /* 2: per-step a/j/s; 1, 3: start-up passes */
    int kind;       /* 0: LDS-tiled kernel; 1: source-parallel small-set kernel;
                       2: evaluation kernel of the device-resident loop (its
                       shape is chosen per block on the device); 4: the
                       loop's finishing kernel (on = 2) */
    int block, ipl; /* launch shape of the instantiation (kind 2: 64, 2;
                       kind 4: 0, 0) */
    int precision;  /* H6_FP64, H6_MIXED, H6_EX or H6_SP */
    int nact_log2;  /* bin: floor(log2(n_act)) of the launches in this record;
                       -1: device-loop launches of blocks with nothing due;
                       -2: prediction slots of the device loop (the
                       finishing kernel predicts every particle to the
                       planned block time; the evaluation does nothing) */
    int64_t launches;
    double interactions; /* sum of n_act * n over the launches (kind 4:
                            those of the blocks they belong to; 0 for
                            prediction slots) */
    double kernel_ms;    /* sum of the event-measured kernel durations */
    double bytes;        /* sum of the launches' algorithmic HBM bytes, each
                            datum moved once: order-2 evaluations 80 B per
                            source + 76 B per target + 72 B per target and
                            slice written; finishing kernel 368 B + 72 B
                            per slice per active particle and 224 B per
                            inactive one (prediction slots: 224 B per
                            particle); 0 for the start-up passes */
} h6_eval_timing;

int h6_profile_enable(h6_ctx ctx, int on);
int h6_profile_read(h6_ctx ctx, h6_eval_timing *out, int max, int *count);
int h6_profile_slots(h6_ctx ctx, int32_t *out, int max, int *count);

/*
 * The self pair (a particle as its own source) contributes nothing; the
 * evaluation kernels either skip it by index or rely on its terms being
 * m eps^-3 times an exact zero. They skip it when eps is below
 * H6_SELF_MASK_EPS_F64 (FP64 pair arithmetic) or H6_SELF_MASK_EPS_F32 (the
 * FP32-range arithmetics H6_MIXED, H6_EX, H6_SP), eps = 0 included; above,
 * the unmasked self term stays an exact zero for masses below
 * H6_SELF_MASK_MASS_F64 or H6_SELF_MASK_MASS_F32 (where m eps^-3 would
 * overflow: larger masses need a larger eps, or units that make them
 * smaller). h6_self_pair_masked returns 1 if the kernels of this precision
 * skip the self pair for this eps, 0 if not; H6_EINVAL for a negative or
 * non-finite eps or an unknown precision. A pure host function: no device
 * work, no context.
 */
#define H6_SELF_MASK_EPS_F64 0x1p-300
#define H6_SELF_MASK_EPS_F32 0x1p-30
#define H6_SELF_MASK_MASS_F64 0x1p124 /* 2^1024 / 2^900 */
#define H6_SELF_MASK_MASS_F32 0x1p38  /* 2^128 / 2^90 */
int h6_self_pair_masked(double eps, int precision);

/* Text of a return code; text of the context's last failure ("" if none). */
const char *h6_strerror(int code);
const char *h6_last_error(h6_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* H6_H */
