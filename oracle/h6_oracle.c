/*
 * Hermite-6 direct N-body oracle: a plain, slow, FP64 CPU implementation.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it. It shares no code, header, table or constant
 * with the HIP library: every formula here is written out independently.
 *
 * What it computes (Goz et al., "Direct N-body code on low-power embedded
 * ARM GPUs", Sec. 3 item list and Sec. 3 "KERNEL OPTIMIZATIONS"):
 *   - the three stages of the 6th-order Hermite scheme: predict, evaluate
 *     acceleration/jerk/snap, correct (Sec. 3, the stage list);
 *   - the evaluation sums over every other particle and skips the self
 *     term (Sec. 3, kernel step iii);
 *   - the time step from the generalized Aarseth criterion, and energy and
 *     angular momentum as accuracy checks (Sec. 3, item 3; Eq. (1));
 *   - block (power-of-two) time steps, which the paper names among the
 *     standard refinements of the direct method (Sec. 2).
 * The pair terms, corrector, interpolation and criterion follow the
 * 6th-order Hermite scheme the paper cites (Nitadori & Makino 2008); the
 * readings taken where the paper is silent are listed in the design notes.
 *
 * Rules kept on purpose: loops only, no intrinsics, IEEE double with no FMA
 * contraction (build with -ffp-contract=off, never -ffast-math), every
 * long sum Neumaier-compensated. OpenMP splits the outer loop over
 * particles i only; each i's sum is sequential, so results do not depend
 * on the thread count.
 *
 * Array layout: vectors are particle-major, [n][3] doubles; masses [n];
 * times and steps are int64 counts of 2^-40 time units.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_TICK_BITS 40

/* ------------------------------------------------------------------ */
/* Neumaier-compensated summation                                      */
/* ------------------------------------------------------------------ */
typedef struct {
    double s, c;
} csum;

static void cs_add(csum *k, double x)
{
    double t = k->s + x;
    if (fabs(k->s) >= fabs(x))
        k->c += (k->s - t) + x;
    else
        k->c += (x - t) + k->s;
    k->s = t;
}

static double cs_val(const csum *k) { return k->s + k->c; }

static double dot3(const double *p, const double *q)
{
    return p[0] * q[0] + p[1] * q[1] + p[2] * q[2];
}

static double norm3(const double *p) { return sqrt(dot3(p, p)); }

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Pair terms                                                          */
/* ------------------------------------------------------------------ */
/*
 * Contribution of source particle j (mass m) to target i, given the
 * relative position r = x_j - x_i, velocity v = v_j - v_i, acceleration
 * a = a_j - a_i and jerk jr = j_j - j_i. Softened (Plummer) potential
 * phi = -m / sqrt(|r|^2 + eps^2).
 *
 * A is the acceleration m r / R^3 with R^2 = |r|^2 + eps^2, and J, S, C are
 * its first, second and third time derivatives along the relative motion
 * (r' = v, v' = a, a' = jr). Writing alpha = (r.v)/R^2,
 * beta = (v.v + r.a)/R^2 + alpha^2 and
 * gamma = (3 v.a + r.jr)/R^2 + alpha (3 beta - 4 alpha^2), differentiation
 * of m r R^-3 gives
 *   J = m v/R^3 - 3 alpha A
 *   S = m a/R^3 - 6 alpha J - 3 beta A
 *   C = m jr/R^3 - 9 alpha S - 9 beta J - 3 gamma A.
 *
 * order 1: A, J.  order 2: A, J, S.  order 3: A, J, S, C.
 * Output arrays for orders not requested are left untouched.
 */
void orc_pair(const double r[3], const double v[3], const double a[3],
              const double jr[3], double m, double eps2, int order,
              double A[3], double J[3], double S[3], double C[3])
{
    double R2 = dot3(r, r) + eps2;
    double Rinv = 1.0 / sqrt(R2);
    double Rinv2 = Rinv * Rinv;
    double mR3 = m * Rinv * Rinv2;
    double alpha = dot3(r, v) * Rinv2;
    int k;
    for (k = 0; k < 3; k++)
        A[k] = mR3 * r[k];
    for (k = 0; k < 3; k++)
        J[k] = mR3 * v[k] - 3.0 * alpha * A[k];
    if (order < 2)
        return;
    double beta = (dot3(v, v) + dot3(r, a)) * Rinv2 + alpha * alpha;
    for (k = 0; k < 3; k++)
        S[k] = mR3 * a[k] - 6.0 * alpha * J[k] - 3.0 * beta * A[k];
    if (order < 3)
        return;
    double gamma = (3.0 * dot3(v, a) + dot3(r, jr)) * Rinv2
                   + alpha * (3.0 * beta - 4.0 * alpha * alpha);
    for (k = 0; k < 3; k++)
        C[k] = mR3 * jr[k] - 9.0 * alpha * S[k] - 9.0 * beta * J[k]
               - 3.0 * gamma * A[k];
}

/*
 * Sum of pair terms on targets i = idx[k] (or i = k when idx is NULL),
 * k < n_i, from all sources j != i of the n particles.
 *   x, v: [n][3] positions and velocities (predicted, all at one time)
 *   a:    [n][3] accelerations, needed for order >= 2
 *   jk:   [n][3] jerks, needed for order 3
 * Outputs A, J (and S, C by order) are [n_i][3].
 * Returns 0, or -1 on bad arguments.
 */
static int forces_impl(int64_t n, const double *x, const double *v,
                       const double *a, const double *jk, const double *m,
                       double eps2, int64_t n_i, const int64_t *idx, int order,
                       int absolute, double *A, double *J, double *S,
                       double *C);

int orc_forces(int64_t n, const double *x, const double *v, const double *a,
               const double *jk, const double *m, double eps2, int64_t n_i,
               const int64_t *idx, int order, double *A, double *J,
               double *S, double *C)
{
    return forces_impl(n, x, v, a, jk, m, eps2, n_i, idx, order, 0, A, J, S,
                       C);
}

/*
 * Same sums of |pair term| per component: sum_j |A_ij|, sum_j |J_ij|, ...
 * The scale against which the rounding error of a sum is measured (a sum
 * evaluated with unit roundoff u is off by at most about n u times it).
 */
int orc_forces_abs(int64_t n, const double *x, const double *v,
                   const double *a, const double *jk, const double *m,
                   double eps2, int64_t n_i, const int64_t *idx, int order,
                   double *A, double *J, double *S, double *C)
{
    return forces_impl(n, x, v, a, jk, m, eps2, n_i, idx, order, 1, A, J, S,
                       C);
}

static int forces_impl(int64_t n, const double *x, const double *v,
                       const double *a, const double *jk, const double *m,
                       double eps2, int64_t n_i, const int64_t *idx, int order,
                       int absolute, double *A, double *J, double *S,
                       double *C)
{
    if (n < 0 || n_i < 0 || !x || !v || !m || !A || !J || order < 1
        || order > 3)
        return -1;
    if (order >= 2 && (!a || !S))
        return -1;
    if (order >= 3 && (!jk || !C))
        return -1;
    int64_t k;
    for (k = 0; k < n_i; k++) {
        int64_t i = idx ? idx[k] : k;
        if (i < 0 || i >= n)
            return -1;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (k = 0; k < n_i; k++) {
        int64_t i = idx ? idx[k] : k;
        csum sum[12];
        memset(sum, 0, sizeof(sum));
        double zero3[3] = {0.0, 0.0, 0.0};
        for (int64_t jj = 0; jj < n; jj++) {
            if (jj == i)
                continue; /* no self interaction */
            double r[3], dv[3], da[3], dj[3];
            double pA[3], pJ[3], pS[3], pC[3];
            for (int c = 0; c < 3; c++) {
                r[c] = x[3 * jj + c] - x[3 * i + c];
                dv[c] = v[3 * jj + c] - v[3 * i + c];
                da[c] = order >= 2 ? a[3 * jj + c] - a[3 * i + c] : 0.0;
                dj[c] = order >= 3 ? jk[3 * jj + c] - jk[3 * i + c] : 0.0;
            }
            orc_pair(r, dv, order >= 2 ? da : zero3, order >= 3 ? dj : zero3,
                     m[jj], eps2, order, pA, pJ, pS, pC);
            for (int c = 0; c < 3; c++) {
                cs_add(&sum[c], absolute ? fabs(pA[c]) : pA[c]);
                cs_add(&sum[3 + c], absolute ? fabs(pJ[c]) : pJ[c]);
                if (order >= 2)
                    cs_add(&sum[6 + c], absolute ? fabs(pS[c]) : pS[c]);
                if (order >= 3)
                    cs_add(&sum[9 + c], absolute ? fabs(pC[c]) : pC[c]);
            }
        }
        for (int c = 0; c < 3; c++) {
            A[3 * k + c] = cs_val(&sum[c]);
            J[3 * k + c] = cs_val(&sum[3 + c]);
            if (order >= 2)
                S[3 * k + c] = cs_val(&sum[6 + c]);
            if (order >= 3)
                C[3 * k + c] = cs_val(&sum[9 + c]);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Predictor                                                           */
/* ------------------------------------------------------------------ */
/*
 * Taylor prediction of every particle over its own interval delta[i]:
 * position to 5th order, velocity to 4th, acceleration to 3rd, using the
 * stored a, j (jerk), s (snap), c (crackle).
 */
void orc_predict(int64_t n, const double *x, const double *v,
                 const double *a, const double *j, const double *s,
                 const double *c, const double *delta, double *xp,
                 double *vp, double *ap)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; i++) {
        double d = delta[i];
        double d2 = d * d, d3 = d2 * d, d4 = d3 * d, d5 = d4 * d;
        for (int k = 0; k < 3; k++) {
            int64_t q = 3 * i + k;
            xp[q] = x[q] + v[q] * d + a[q] * d2 / 2.0 + j[q] * d3 / 6.0
                    + s[q] * d4 / 24.0 + c[q] * d5 / 120.0;
            vp[q] = v[q] + a[q] * d + j[q] * d2 / 2.0 + s[q] * d3 / 6.0
                    + c[q] * d4 / 24.0;
            ap[q] = a[q] + j[q] * d + s[q] * d2 / 2.0 + c[q] * d3 / 6.0;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Corrector and interpolation                                         */
/* ------------------------------------------------------------------ */
/*
 * Sixth-order corrector over a step of length h, given the acceleration,
 * jerk and snap at both ends (0: old, 1: newly evaluated). The velocity is
 * the two-point Hermite quadrature of a(t) using a, a', a'' at both ends,
 *   v1 = v0 + h/2 (a0+a1) - h^2/10 (j1-j0) + h^3/120 (s0+s1),
 * which is exact when a(t) is a quintic; the position applies the same
 * rule to v(t), whose derivatives are a and j:
 *   x1 = x0 + h/2 (v0+v1) - h^2/10 (a1-a0) + h^3/120 (j0+j1).
 *
 * Interpolation: the quintic matching a, j, s at both ends is differenced
 * to give crackle, pop and the fifth derivative at the end of the step:
 *   c1  = [  60 (a1-a0) - h (24 j0 + 36 j1)   + h^2 (9 s1 - 3 s0)  ] / h^3
 *   p1  = [ 360 (a1-a0) - h (168 j0 + 192 j1) + h^2 (36 s1 - 24 s0) ] / h^4
 *   d5a = [ 720 (a1-a0) - 360 h (j0 + j1)     + 60 h^2 (s1 - s0)   ] / h^5
 * All arrays are [n][3]; h is per particle.
 */
void orc_correct(int64_t n, const double *x0, const double *v0,
                 const double *a0, const double *j0, const double *s0,
                 const double *a1, const double *j1, const double *s1,
                 const double *h, double *x1, double *v1, double *c1,
                 double *p1, double *d5a)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; i++) {
        double dt = h[i];
        double dt2 = dt * dt, dt3 = dt2 * dt, dt4 = dt3 * dt, dt5 = dt4 * dt;
        for (int k = 0; k < 3; k++) {
            int64_t q = 3 * i + k;
            double vn = v0[q] + dt / 2.0 * (a0[q] + a1[q])
                        - dt2 / 10.0 * (j1[q] - j0[q])
                        + dt3 / 120.0 * (s0[q] + s1[q]);
            double xn = x0[q] + dt / 2.0 * (v0[q] + vn)
                        - dt2 / 10.0 * (a1[q] - a0[q])
                        + dt3 / 120.0 * (j0[q] + j1[q]);
            double da = a1[q] - a0[q];
            v1[q] = vn;
            x1[q] = xn;
            c1[q] = (60.0 * da - dt * (24.0 * j0[q] + 36.0 * j1[q])
                     + dt2 * (9.0 * s1[q] - 3.0 * s0[q])) / dt3;
            if (p1)
                p1[q] = (360.0 * da - dt * (168.0 * j0[q] + 192.0 * j1[q])
                         + dt2 * (36.0 * s1[q] - 24.0 * s0[q])) / dt4;
            if (d5a)
                d5a[q] = (720.0 * da - 360.0 * dt * (j0[q] + j1[q])
                          + 60.0 * dt2 * (s1[q] - s0[q])) / dt5;
        }
    }
}

/* ------------------------------------------------------------------ */
/* Time-step criteria                                                  */
/* ------------------------------------------------------------------ */
/*
 * Generalized Aarseth criterion of order 6:
 *   dt = eta * [ (|a||s| + |j|^2) / (|c||d5a| + |p|^2) ]^(1/6).
 * (The general member is (A(1)/A(p-2))^(1/(2(p-3))) with
 * A(k) = |a^(k-1)||a^(k+1)| + |a^(k)|^2; p = 6 here.)
 */
double orc_dt_crit6(const double *a, const double *j, const double *s,
                    const double *c, const double *p, const double *d5a,
                    double eta)
{
    double num = norm3(a) * norm3(s) + dot3(j, j);
    double den = norm3(c) * norm3(d5a) + dot3(p, p);
    return eta * pow(num / den, 1.0 / 6.0);
}

/* Start-up criterion, the p = 4 member: eta_s [(|a||s|+|j|^2)/(|j||c|+|s|^2)]^(1/2). */
double orc_dt_crit4(const double *a, const double *j, const double *s,
                    const double *c, double eta_s)
{
    double num = norm3(a) * norm3(s) + dot3(j, j);
    double den = norm3(j) * norm3(c) + dot3(s, s);
    return eta_s * sqrt(num / den);
}

/* Smallest level L >= lev_min with 2^-L <= dt (dt = +inf gives lev_min). */
int orc_level_of(double dt, int lev_min, int lev_cap)
{
    int lev = lev_min;
    while (lev <= lev_cap && ldexp(1.0, -lev) > dt)
        lev++;
    return lev;
}

/*
 * Power-of-two block-step rule. A step may shrink by any number of levels;
 * it may grow by one level only, and only when the new time t1 is a
 * multiple of twice the old step (so that the particle stays in step with
 * the coarser block).
 */
int orc_next_level(int lev_old, int lev_crit, int64_t t1_ticks)
{
    if (lev_crit > lev_old)
        return lev_crit;
    if (lev_crit < lev_old) {
        int64_t two_old = (int64_t)1 << (ORC_TICK_BITS - lev_old + 1);
        if (t1_ticks % two_old == 0)
            return lev_old - 1;
    }
    return lev_old;
}

static int64_t level_ticks(int lev)
{
    return (int64_t)1 << (ORC_TICK_BITS - lev);
}

static double ticks_to_time(int64_t t)
{
    return ldexp((double)t, -ORC_TICK_BITS);
}

/* ------------------------------------------------------------------ */
/* Start-up                                                            */
/* ------------------------------------------------------------------ */
/*
 * No snap or crackle exist at t = 0. Pass 1 evaluates a and j from x, v;
 * pass 2 evaluates s and c with the pass-1 a and j of every particle as
 * the sources' acceleration and jerk.
 */
int orc_startup(int64_t n, const double *x, const double *v, const double *m,
                double eps2, double *a, double *j, double *s, double *c)
{
    int rc = orc_forces(n, x, v, NULL, NULL, m, eps2, n, NULL, 1, a, j, NULL,
                        NULL);
    if (rc)
        return rc;
    double *a2 = malloc(sizeof(double) * 3 * (size_t)(n ? n : 1));
    double *j2 = malloc(sizeof(double) * 3 * (size_t)(n ? n : 1));
    if (!a2 || !j2) {
        free(a2);
        free(j2);
        return -2;
    }
    rc = orc_forces(n, x, v, a, j, m, eps2, n, NULL, 3, a2, j2, s, c);
    free(a2);
    free(j2);
    return rc;
}

/* Initial levels from the start-up criterion; returns -5 if below lev_max. */
int orc_initial_levels(int64_t n, const double *a, const double *j,
                       const double *s, const double *c, double eta_s,
                       int lev_min, int lev_max, int64_t *dt_ticks)
{
    int bad = 0;
    for (int64_t i = 0; i < n; i++) {
        double d = orc_dt_crit4(a + 3 * i, j + 3 * i, s + 3 * i, c + 3 * i,
                                eta_s);
        int lev = orc_level_of(d, lev_min, lev_max + 1);
        if (lev > lev_max) {
            bad = 1;
            lev = lev_max;
        }
        dt_ticks[i] = level_ticks(lev);
    }
    return bad ? -5 : 0;
}

/* ------------------------------------------------------------------ */
/* Block scheduling                                                    */
/* ------------------------------------------------------------------ */
/* Next block time min(t+dt) and the particles due then, in index order. */
int64_t orc_next_block(int64_t n, const int64_t *t, const int64_t *dt,
                       int64_t *active, int64_t *n_act)
{
    int64_t tn = INT64_MAX;
    for (int64_t i = 0; i < n; i++)
        if (t[i] + dt[i] < tn)
            tn = t[i] + dt[i];
    int64_t k = 0;
    for (int64_t i = 0; i < n; i++)
        if (t[i] + dt[i] == tn)
            active[k++] = i;
    *n_act = k;
    return tn;
}

/* ------------------------------------------------------------------ */
/* Integrator steps                                                    */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t n;
    double *x, *v, *a, *j, *s, *c, *m; /* [n][3], m [n] */
    int64_t *t, *dt;                   /* ticks */
} orc_state;

static void *xmalloc(size_t bytes) { return malloc(bytes ? bytes : 1); }

/*
 * One block step: select the block, predict every particle to its time,
 * evaluate a, j, s on the active particles, correct them, interpolate
 * crackle (kept for the next prediction), pop and the fifth derivative,
 * and assign new power-of-two steps.
 * Returns 0, -2 (memory) or -5 (a step fell below 2^-lev_max; the state
 * is still advanced with the step clamped at lev_max).
 */
int orc_block_step(orc_state *st, double eps2, double eta, int lev_min,
                   int lev_max, int64_t *t_next_out, int64_t *n_act_out)
{
    int64_t n = st->n;
    size_t v3 = sizeof(double) * 3 * (size_t)n;
    int64_t *act = xmalloc(sizeof(int64_t) * (size_t)n);
    double *delta = xmalloc(sizeof(double) * (size_t)n);
    double *xp = xmalloc(v3), *vp = xmalloc(v3), *ap = xmalloc(v3);
    double *f = xmalloc(9 * sizeof(double) * (size_t)n);
    double *o = xmalloc(33 * sizeof(double) * (size_t)n);
    double *hh = xmalloc(sizeof(double) * (size_t)n);
    int rc = 0;
    if (!act || !delta || !xp || !vp || !ap || !f || !o || !hh) {
        rc = -2;
        goto done;
    }
    int64_t n_act;
    int64_t tn = orc_next_block(n, st->t, st->dt, act, &n_act);
    for (int64_t i = 0; i < n; i++)
        delta[i] = ticks_to_time(tn - st->t[i]);
    orc_predict(n, st->x, st->v, st->a, st->j, st->s, st->c, delta, xp, vp,
                ap);
    double *A1 = f, *J1 = f + 3 * n_act, *S1 = f + 6 * n_act;
    rc = orc_forces(n, xp, vp, ap, NULL, st->m, eps2, n_act, act, 2, A1, J1,
                    S1, NULL);
    if (rc)
        goto done;
    /* gather the old state of the active particles */
    double *X0 = o, *V0 = o + 3 * n_act, *Ao = o + 6 * n_act,
           *Jo = o + 9 * n_act, *So = o + 12 * n_act;
    double *X1 = o + 15 * n_act, *Vn = o + 18 * n_act, *Cn = o + 21 * n_act,
           *Pn = o + 24 * n_act, *Dn = o + 27 * n_act;
    for (int64_t k = 0; k < n_act; k++) {
        int64_t i = act[k];
        memcpy(X0 + 3 * k, st->x + 3 * i, 3 * sizeof(double));
        memcpy(V0 + 3 * k, st->v + 3 * i, 3 * sizeof(double));
        memcpy(Ao + 3 * k, st->a + 3 * i, 3 * sizeof(double));
        memcpy(Jo + 3 * k, st->j + 3 * i, 3 * sizeof(double));
        memcpy(So + 3 * k, st->s + 3 * i, 3 * sizeof(double));
        hh[k] = ticks_to_time(st->dt[i]);
    }
    orc_correct(n_act, X0, V0, Ao, Jo, So, A1, J1, S1, hh, X1, Vn, Cn, Pn,
                Dn);
    for (int64_t k = 0; k < n_act; k++) {
        int64_t i = act[k];
        memcpy(st->x + 3 * i, X1 + 3 * k, 3 * sizeof(double));
        memcpy(st->v + 3 * i, Vn + 3 * k, 3 * sizeof(double));
        memcpy(st->a + 3 * i, A1 + 3 * k, 3 * sizeof(double));
        memcpy(st->j + 3 * i, J1 + 3 * k, 3 * sizeof(double));
        memcpy(st->s + 3 * i, S1 + 3 * k, 3 * sizeof(double));
        memcpy(st->c + 3 * i, Cn + 3 * k, 3 * sizeof(double));
        double d = orc_dt_crit6(A1 + 3 * k, J1 + 3 * k, S1 + 3 * k,
                                Cn + 3 * k, Pn + 3 * k, Dn + 3 * k, eta);
        int lc = orc_level_of(d, lev_min, lev_max + 1);
        int lo = ORC_TICK_BITS;
        while (lo > 0 && level_ticks(lo) != st->dt[i])
            lo--;
        int ln = orc_next_level(lo, lc, tn);
        if (ln > lev_max) {
            rc = -5;
            ln = lev_max;
        }
        st->t[i] = tn;
        st->dt[i] = level_ticks(ln);
    }
    *t_next_out = tn;
    *n_act_out = n_act;
done:
    free(act);
    free(delta);
    free(xp);
    free(vp);
    free(ap);
    free(f);
    free(o);
    free(hh);
    return rc;
}

/* Flat-argument wrapper of orc_block_step for foreign callers. */
int orc_block_step_flat(int64_t n, double *x, double *v, double *a,
                        double *j, double *s, double *c, double *m,
                        int64_t *t, int64_t *dt, double eps2, double eta,
                        int lev_min, int lev_max, int64_t *t_next,
                        int64_t *n_act)
{
    orc_state st = {n, x, v, a, j, s, c, m, t, dt};
    return orc_block_step(&st, eps2, eta, lev_min, lev_max, t_next, n_act);
}

/*
 * nsteps shared steps of length h: every particle is predicted, evaluated
 * and corrected each step; crackle is interpolated for the next
 * prediction. No step-size logic.
 */
int orc_shared_steps(int64_t n, double *x, double *v, double *a, double *j,
                     double *s, double *c, const double *m, double eps2,
                     double h, int64_t nsteps)
{
    size_t v3 = sizeof(double) * 3 * (size_t)n;
    double *delta = xmalloc(sizeof(double) * (size_t)n);
    double *xp = xmalloc(v3), *vp = xmalloc(v3), *ap = xmalloc(v3);
    double *A1 = xmalloc(v3), *J1 = xmalloc(v3), *S1 = xmalloc(v3);
    int rc = 0;
    if (!delta || !xp || !vp || !ap || !A1 || !J1 || !S1) {
        rc = -2;
        goto done;
    }
    for (int64_t i = 0; i < n; i++)
        delta[i] = h;
    for (int64_t st = 0; st < nsteps; st++) {
        orc_predict(n, x, v, a, j, s, c, delta, xp, vp, ap);
        rc = orc_forces(n, xp, vp, ap, NULL, m, eps2, n, NULL, 2, A1, J1, S1,
                        NULL);
        if (rc)
            goto done;
        orc_correct(n, x, v, a, j, s, A1, J1, S1, delta, x, v, c, NULL,
                    NULL);
        memcpy(a, A1, v3);
        memcpy(j, J1, v3);
        memcpy(s, S1, v3);
    }
done:
    free(delta);
    free(xp);
    free(vp);
    free(ap);
    free(A1);
    free(J1);
    free(S1);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Energy and angular momentum (accuracy diagnostics, Eq. (1))         */
/* ------------------------------------------------------------------ */
/*
 * out[0] kinetic energy sum m|v|^2/2; out[1] potential energy
 * -sum_{i<j} m_i m_j / sqrt(|x_i-x_j|^2 + eps^2); out[2..4] angular
 * momentum sum m x cross v. Every sum compensated.
 */
int orc_energy(int64_t n, const double *x, const double *v, const double *m,
               double eps2, double *out)
{
    double *phi = xmalloc(sizeof(double) * (size_t)n);
    if (!phi)
        return -2;
    int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < n; i++) {
        csum p = {0.0, 0.0};
        for (int64_t jj = i + 1; jj < n; jj++) {
            double r[3];
            for (int c = 0; c < 3; c++)
                r[c] = x[3 * jj + c] - x[3 * i + c];
            cs_add(&p, m[jj] / sqrt(dot3(r, r) + eps2));
        }
        phi[i] = m[i] * cs_val(&p);
    }
    csum ek = {0, 0}, ep = {0, 0}, L[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (i = 0; i < n; i++) {
        const double *xi = x + 3 * i, *vi = v + 3 * i;
        cs_add(&ek, 0.5 * m[i] * dot3(vi, vi));
        cs_add(&ep, -phi[i]);
        cs_add(&L[0], m[i] * (xi[1] * vi[2] - xi[2] * vi[1]));
        cs_add(&L[1], m[i] * (xi[2] * vi[0] - xi[0] * vi[2]));
        cs_add(&L[2], m[i] * (xi[0] * vi[1] - xi[1] * vi[0]));
    }
    out[0] = cs_val(&ek);
    out[1] = cs_val(&ep);
    for (int c = 0; c < 3; c++)
        out[2 + c] = cs_val(&L[c]);
    free(phi);
    return 0;
}

/*
 * Potential of each particle (the per-particle terms of the energy of
 * Sec. 3 item 3): phi[i] = -sum_{j != i} m_j / sqrt(|x_j - x_i|^2 + eps^2),
 * compensated. sum_i m_i phi[i] / 2 is the potential energy.
 */
int orc_potential(int64_t n, const double *x, const double *m, double eps2, double *phi)
{
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < n; i++) {
        csum p = {0.0, 0.0};
        for (int64_t jj = 0; jj < n; jj++) {
            if (jj == i)
                continue;
            double r[3];
            for (int c = 0; c < 3; c++)
                r[c] = x[3 * jj + c] - x[3 * i + c];
            cs_add(&p, m[jj] / sqrt(dot3(r, r) + eps2));
        }
        phi[i] = -cs_val(&p);
    }
    return 0;
}
