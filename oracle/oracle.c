/*
 * oracle.c -- plain CPU reference for the swept-rule hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this file; only the tests, the package smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no source with the HIP
 * path.
 *
 * What it computes.  The swept rule reorders the work of an explicit scheme
 * but applies the same numerical method as classic step-by-step stepping and
 * performs no redundant operation (Magee, Walker & Niemeyer, Sec. 2 and
 * Sec. 4.1).  The plain definition of the swept result is therefore classic
 * periodic time stepping of the two test schemes, which is what this file
 * does: every stage is applied to every cell before the next stage starts,
 * with whole-array temporaries, in plain scalar loops.
 *
 *   heat  : first-order forward-in-time, central-in-space (Sec. 4.2)
 *   euler : second-order finite volume with a minmod limiter (Sec. 4.2),
 *           organised as four three-point sub-steps per time step with a
 *           stored pressure ratio (the "lengthening" layout, Sec. 4.3,
 *           Fig. 2b): Pr(Q0) -> predictor -> Pr(Q1) -> corrector.
 *   ks    : the Kuramoto-Sivashinsky equation, which the paper names (Sec. 2)
 *           among the equations the swept rule has been applied to; forward
 *           Euler in time, central differences, a five-point stencil.
 *
 * The paper defers the exact scheme equations to an earlier article; the
 * reading used here (textbook FTCS; pressure-ratio minmod reconstruction,
 * Rusanov flux, midpoint predictor-corrector, gamma = 1.4) is written out in
 * the functions below and every operation is evaluated in exactly the
 * written parenthesisation.  Build with -ffp-contract=off and without
 * fast-math: no fused multiply-add, IEEE division and square root.
 *
 * Two precisions:
 *   *_f64 : everything in binary64 (the reference result).
 *   *_f32 : the single-precision variant of the same schemes -- binary32
 *           state and flux arithmetic, Kahan-compensated accumulation of the
 *           time update, binary64 for the pressure / velocity / sound-speed
 *           recovery, the pressure ratio and the limiter value.  It mirrors
 *           the precision pattern of the GPU single-precision path operation
 *           for operation, so that path can be checked bit for bit.
 *
 * OpenMP splits the cell loops; there are no reductions, so the result is
 * bit-identical for any thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GAMMA 1.4 /* ratio of specific heats, as a binary64 literal */
#define GM1 0.4   /* gamma - 1 as its own literal (1.4 - 1.0 rounds differently) */

static int64_t wrap(int64_t i, int64_t n)
{
    int64_t r = i % n;
    return r < 0 ? r + n : r;
}

static void set_threads(int threads)
{
#ifdef _OPENMP
    if (threads > 0)
        omp_set_num_threads(threads);
#else
    (void)threads;
#endif
}

int oracle_threads_used(int threads)
{
#ifdef _OPENMP
    if (threads > 0)
        return threads;
    return omp_get_max_threads();
#else
    (void)threads;
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Heat equation, FTCS (Sec. 4.2).
 *   u_i^{n+1} = u_i^n + r * ((u_{i+1}^n - u_i^n) + (u_{i-1}^n - u_i^n)),
 *   r = alpha*dt/dx^2, periodic indices.
 * ---------------------------------------------------------------------- */
int oracle_heat_f64(double *u, int64_t n, int64_t steps, double r, int threads)
{
    if (n < 3 || steps < 0 || !u)
        return 1;
    double *v = (double *)malloc((size_t)n * sizeof(double));
    if (!v)
        return 4;
    set_threads(threads);
    double *cur = u, *nxt = v;
    for (int64_t s = 0; s < steps; ++s) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double left = cur[wrap(i - 1, n)];
            double mid = cur[i];
            double right = cur[wrap(i + 1, n)];
            nxt[i] = mid + r * ((right - mid) + (left - mid));
        }
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != u)
        memcpy(u, cur, (size_t)n * sizeof(double));
    free(v);
    return 0;
}

/* Same scheme with binary32 state; the increment is accumulated with Kahan
 * compensation (c holds the running compensation, carried between calls). */
int oracle_heat_f32(float *u, float *c, int64_t n, int64_t steps, float r, int threads)
{
    if (n < 3 || steps < 0 || !u || !c)
        return 1;
    float *v = (float *)malloc((size_t)n * sizeof(float));
    if (!v)
        return 4;
    set_threads(threads);
    float *cur = u, *nxt = v;
    for (int64_t s = 0; s < steps; ++s) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            float left = cur[wrap(i - 1, n)];
            float mid = cur[i];
            float right = cur[wrap(i + 1, n)];
            float delta = r * ((right - mid) + (left - mid));
            float y = delta - c[i];
            float t = mid + y;
            c[i] = (t - mid) - y;
            nxt[i] = t;
        }
        float *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != u)
        memcpy(u, cur, (size_t)n * sizeof(float));
    free(v);
    return 0;
}

/* ------------------------------------------------------------------------
 * Euler equations, binary64.
 * Conserved U = (rho, m = rho*u, E).  Pressure from the ideal-gas law.
 * ---------------------------------------------------------------------- */

/* velocity and pressure of a conserved state */
static void prim64(double rho, double m, double e, double *vel, double *p)
{
    double uu = m / rho;
    *vel = uu;
    *p = GM1 * (e - 0.5 * (m * uu));
}

/* minmod limiter in ratio form: phi(q) = max(0, min(q, 1)); NaN -> 0 */
static double limiter64(double q)
{
    if (q > 0.0)
        return q < 1.0 ? q : 1.0;
    return 0.0;
}

/* pressure ratio of cell i: forward over backward pressure difference */
static double pratio64(double pm, double pc, double pp)
{
    return (pp - pc) / (pc - pm);
}

/* Rusanov flux at the face between cell L (state a, ratio pra) and cell R
 * (state b, ratio prb); a and b point at (rho, m, E). */
static void face_flux64(const double a[3], const double b[3], double pra, double prb,
                        double f[3])
{
    double phil = limiter64(1.0 / pra); /* backward/forward ratio of cell L */
    double phir = limiter64(prb);       /* forward/backward ratio of cell R */
    double ul[3], ur[3];
    for (int k = 0; k < 3; ++k) {
        double d = b[k] - a[k];
        ul[k] = a[k] + (0.5 * phil) * d;
        ur[k] = b[k] - (0.5 * phir) * d;
    }
    double vl, pl, vr, pr;
    prim64(ul[0], ul[1], ul[2], &vl, &pl);
    prim64(ur[0], ur[1], ur[2], &vr, &pr);
    double al = sqrt((GAMMA * pl) / ul[0]);
    double ar = sqrt((GAMMA * pr) / ur[0]);
    double fl[3] = {ul[1], ul[1] * vl + pl, (ul[2] + pl) * vl};
    double fr[3] = {ur[1], ur[1] * vr + pr, (ur[2] + pr) * vr};
    double sl = fabs(vl) + al;
    double sr = fabs(vr) + ar;
    double sig = sl > sr ? sl : sr;
    for (int k = 0; k < 3; ++k)
        f[k] = 0.5 * (fl[k] + fr[k]) - (0.5 * sig) * (ur[k] - ul[k]);
}

/* Pressure-ratio sub-step over the whole grid from the states q[3][n]. */
static void pr_stage64(const double *q0, const double *q1, const double *q2, double *p,
                       double *pr, int64_t n)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double vel;
        prim64(q0[i], q1[i], q2[i], &vel, &p[i]);
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        pr[i] = pratio64(p[wrap(i - 1, n)], p[i], p[wrap(i + 1, n)]);
}

/* Face fluxes of the whole grid: f[k][i] is the flux through the face
 * between cell i-1 and cell i. */
static void flux_stage64(double *const q[3], const double *pr, double *const f[3], int64_t n)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t l = wrap(i - 1, n);
        double a[3] = {q[0][l], q[1][l], q[2][l]};
        double b[3] = {q[0][i], q[1][i], q[2][i]};
        double ff[3];
        face_flux64(a, b, pr[l], pr[i], ff);
        f[0][i] = ff[0];
        f[1][i] = ff[1];
        f[2][i] = ff[2];
    }
}

/* state arrays: rho, m, E of length n, updated in place; lam = dt/dx */
int oracle_euler_f64(double *rho, double *mom, double *ene, int64_t n, int64_t steps,
                     double lam, int threads)
{
    if (n < 3 || steps < 0 || !rho || !mom || !ene)
        return 1;
    double *buf = (double *)malloc((size_t)n * 8 * sizeof(double));
    if (!buf)
        return 4;
    set_threads(threads);
    double *q0[3] = {rho, mom, ene};
    double *q1[3] = {buf, buf + n, buf + 2 * n};
    double *f[3] = {buf + 3 * n, buf + 4 * n, buf + 5 * n};
    double *p = buf + 6 * n, *pr = buf + 7 * n;
    double half_lam = 0.5 * lam;
    for (int64_t s = 0; s < steps; ++s) {
        /* sub-step 1: pressure ratio of the time-level state */
        pr_stage64(q0[0], q0[1], q0[2], p, pr, n);
        /* sub-step 2: predictor to the half step */
        flux_stage64(q0, pr, f, n);
        for (int k = 0; k < 3; ++k) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i)
                q1[k][i] = q0[k][i] + half_lam * (f[k][i] - f[k][wrap(i + 1, n)]);
        }
        /* sub-step 3: pressure ratio of the predicted state */
        pr_stage64(q1[0], q1[1], q1[2], p, pr, n);
        /* sub-step 4: corrector, full step with half-step fluxes */
        flux_stage64(q1, pr, f, n);
        for (int k = 0; k < 3; ++k) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i)
                q0[k][i] = q0[k][i] + lam * (f[k][i] - f[k][wrap(i + 1, n)]);
        }
    }
    free(buf);
    return 0;
}

/* ------------------------------------------------------------------------
 * Euler equations, binary32 state with binary64 islands.
 * ---------------------------------------------------------------------- */

/* pressure of a binary32 state, evaluated in binary64 */
static double pres32(float rho, float m, float e)
{
    double dr = (double)rho, dm = (double)m, de = (double)e;
    double uu = dm / dr;
    return GM1 * (de - 0.5 * (dm * uu));
}

static void face_flux32(const float a[3], const float b[3], double pra, double prb, float f[3])
{
    float hl = 0.5f * (float)limiter64(1.0 / pra);
    float hr = 0.5f * (float)limiter64(prb);
    float ul[3], ur[3];
    for (int k = 0; k < 3; ++k) {
        float d = b[k] - a[k];
        ul[k] = a[k] + hl * d;
        ur[k] = b[k] - hr * d;
    }
    /* recovery of velocity, pressure and sound speed in binary64 */
    double rl = (double)ul[0], ml = (double)ul[1], el = (double)ul[2];
    double rr = (double)ur[0], mr = (double)ur[1], er = (double)ur[2];
    double vl64 = ml / rl, vr64 = mr / rr;
    double pl64 = GM1 * (el - 0.5 * (ml * vl64));
    double pr64 = GM1 * (er - 0.5 * (mr * vr64));
    double al64 = sqrt((GAMMA * pl64) / rl);
    double ar64 = sqrt((GAMMA * pr64) / rr);
    float vl = (float)vl64, pl = (float)pl64, al = (float)al64;
    float vr = (float)vr64, pr = (float)pr64, ar = (float)ar64;
    float fl[3] = {ul[1], ul[1] * vl + pl, (ul[2] + pl) * vl};
    float fr[3] = {ur[1], ur[1] * vr + pr, (ur[2] + pr) * vr};
    float sl = fabsf(vl) + al;
    float sr = fabsf(vr) + ar;
    float sig = sl > sr ? sl : sr;
    for (int k = 0; k < 3; ++k)
        f[k] = 0.5f * (fl[k] + fr[k]) - (0.5f * sig) * (ur[k] - ul[k]);
}

static void pr_stage32(float *const q[3], double *p, double *pr, int64_t n)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        p[i] = pres32(q[0][i], q[1][i], q[2][i]);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        pr[i] = pratio64(p[wrap(i - 1, n)], p[i], p[wrap(i + 1, n)]);
}

static void flux_stage32(float *const q[3], const double *pr, float *const f[3], int64_t n)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t l = wrap(i - 1, n);
        float a[3] = {q[0][l], q[1][l], q[2][l]};
        float b[3] = {q[0][i], q[1][i], q[2][i]};
        float ff[3];
        face_flux32(a, b, pr[l], pr[i], ff);
        f[0][i] = ff[0];
        f[1][i] = ff[1];
        f[2][i] = ff[2];
    }
}

/* state: rho, m, E and their Kahan compensations crho, cm, cE (binary32) */
int oracle_euler_f32(float *rho, float *mom, float *ene, float *crho, float *cmom,
                     float *cene, int64_t n, int64_t steps, float lam, int threads)
{
    if (n < 3 || steps < 0 || !rho || !mom || !ene || !crho || !cmom || !cene)
        return 1;
    float *fb = (float *)malloc((size_t)n * 6 * sizeof(float));
    double *db = (double *)malloc((size_t)n * 2 * sizeof(double));
    if (!fb || !db) {
        free(fb);
        free(db);
        return 4;
    }
    set_threads(threads);
    float *q0[3] = {rho, mom, ene};
    float *cc[3] = {crho, cmom, cene};
    float *q1[3] = {fb, fb + n, fb + 2 * n};
    float *f[3] = {fb + 3 * n, fb + 4 * n, fb + 5 * n};
    double *p = db, *pr = db + n;
    float half_lam = 0.5f * lam;
    for (int64_t s = 0; s < steps; ++s) {
        pr_stage32(q0, p, pr, n);
        flux_stage32(q0, pr, f, n);
        for (int k = 0; k < 3; ++k) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i)
                q1[k][i] = q0[k][i] + half_lam * (f[k][i] - f[k][wrap(i + 1, n)]);
        }
        pr_stage32(q1, p, pr, n);
        flux_stage32(q1, pr, f, n);
        for (int k = 0; k < 3; ++k) {
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < n; ++i) {
                float delta = lam * (f[k][i] - f[k][wrap(i + 1, n)]);
                float y = delta - cc[k][i];
                float t = q0[k][i] + y;
                cc[k][i] = (t - q0[k][i]) - y;
                q0[k][i] = t;
            }
        }
    }
    free(fb);
    free(db);
    return 0;
}

/* ------------------------------------------------------------------------
 * Kuramoto-Sivashinsky equation  u_t + u u_x + u_xx + u_xxxx = 0
 * (named in Sec. 2 among the equations the swept rule has been applied
 * to; the paper gives no scheme).  Reading: forward Euler in time, the
 * advection in conservative form with a central difference of the flux
 * u^2/2, the second derivative as the difference form of the heat scheme
 * and the fourth derivative as the same second difference applied to the
 * second differences.  Per time step, each stage over every cell before
 * the next:
 *   s_i  = (u_{i+1} - u_i) + (u_{i-1} - u_i)
 *   f_i  = 0.5 * (u_i * u_i)
 *   q_i  = (s_{i+1} - s_i) + (s_{i-1} - s_i)
 *   u_i <- u_i - ((a * (f_{i+1} - f_{i-1}) + b * s_i) + c * q_i)
 * with a = dt / (2 dx), b = dt / dx^2, c = dt / dx^4 (passed in).
 * ---------------------------------------------------------------------- */
int oracle_ks_f64(double *u, int64_t n, int64_t steps, double a, double b, double c,
                  int threads)
{
    if (n < 5 || steps < 0 || !u)
        return 1;
    double *s2 = (double *)malloc((size_t)n * sizeof(double));
    double *fl = (double *)malloc((size_t)n * sizeof(double));
    double *q4 = (double *)malloc((size_t)n * sizeof(double));
    if (!s2 || !fl || !q4) {
        free(s2);
        free(fl);
        free(q4);
        return 4;
    }
    set_threads(threads);
    for (int64_t st = 0; st < steps; ++st) {
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            const double mid = u[i];
            s2[i] = (u[wrap(i + 1, n)] - mid) + (u[wrap(i - 1, n)] - mid);
            fl[i] = 0.5 * (mid * mid);
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            const double mid = s2[i];
            q4[i] = (s2[wrap(i + 1, n)] - mid) + (s2[wrap(i - 1, n)] - mid);
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i)
            u[i] = u[i] - ((a * (fl[wrap(i + 1, n)] - fl[wrap(i - 1, n)]) + b * s2[i]) + c * q4[i]);
    }
    free(s2);
    free(fl);
    free(q4);
    return 0;
}
