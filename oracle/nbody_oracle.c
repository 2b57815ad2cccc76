/*
 * FP64 reference oracle for direct-summation N-body forces and the Hermite
 * block-step integrator.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file: only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or helper with
 * the GPU library.  It is written to be read against the paper, not to be
 * fast: plain double loops, IEEE binary64, round to nearest, no fast-math,
 * j visited in ascending order.  The only parallelism is an optional
 * OpenMP split over the outer (independent) i loop, which does not change
 * any result.
 *
 * Layout: a vector field over n particles is three contiguous rows of n
 * doubles (all x, then all y, then all z).  Times and time steps are int64
 * ticks of 2^-20 N-body time units.
 *
 * What is computed, and where it comes from:
 *  - Eq. 1 (Section 2): Newtonian acceleration by direct summation over
 *    j != i.  The printed sign (r_i - r_j) would be repulsive; the oracle
 *    uses the attractive direction r_ij = r_j - r_i (pinned by a = -grad phi
 *    with phi < 0 and by the two-body closed form).
 *  - Plummer softening (Section 3.3, after Aarseth 1963): r^2 -> r^2 + eps^2
 *    in acceleration, jerk and potential.
 *  - Jerk (Section 3, the Hermite scheme needs da/dt) and potential
 *    (Section 3.1, the self interaction is removed): jerk is the time
 *    derivative of the softened acceleration along the particle velocities;
 *    phi_i = -G sum_{j != i} m_j / sqrt(r^2 + eps^2).  Self is excluded by
 *    index, never by r = 0.  With eps = 0, a pair at zero separation is
 *    skipped (Section 3.3, the zero-softening check).
 *  - Fourth-order Hermite predictor-corrector (Section 3, Makino & Aarseth
 *    1992) with one force evaluation per step, and block (hierarchical,
 *    power-of-two) time steps (Section 3.1, Makino 1991).
 *  - Energy (Eq. 2, Section 4): E = sum m v^2 / 2 + sum m phi / 2.
 *  - Adjoint (vector-Jacobian product) of the force with respect to
 *    positions, velocities and masses, and of a shared-step Hermite run.
 *
 * The paper prints none of the Hermite, time-step or jerk formulas; the
 * readings taken are listed in the design notes and restated beside each
 * function below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TICK (1.0 / 1048576.0) /* one tick = 2^-20 time units */

static void set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------
 * Force: acceleration, jerk and potential of i-particles from j-particles.
 *
 * For each i, for j = 0 .. nj-1 in order, skipping j == iself[i]:
 *   r = x_j - x_i,  u = v_j - v_i,  s = r.r + eps^2
 *   A = s^-1/2,  B = A^3,  C = A^5
 *   a_i    += G m_j B r
 *   jerk_i += G m_j (B u - 3 C (r.u) r)
 *   phi_i  -= G m_j A
 * iself may be NULL (no exclusion).  With eps == 0 a pair with s == 0 is
 * skipped.  Outputs are overwritten.
 * ---------------------------------------------------------------------- */
int oracle_force(int64_t ni, const double *xi, const double *vi, const int64_t *iself,
                 int64_t nj, const double *xj, const double *vj, const double *mj,
                 double G, double eps, double *acc, double *jerk, double *pot,
                 int nthreads) {
    if (ni < 0 || nj < 0 || eps < 0) return -1;
    set_threads(nthreads);
    const double eps2 = eps * eps;
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < ni; ++i) {
        const double px = xi[i], py = xi[ni + i], pz = xi[2 * ni + i];
        const double qx = vi[i], qy = vi[ni + i], qz = vi[2 * ni + i];
        double ax = 0, ay = 0, az = 0, jx = 0, jy = 0, jz = 0, ph = 0;
        const int64_t self = iself ? iself[i] : -1;
        for (int64_t j = 0; j < nj; ++j) {
            if (j == self) continue;
            const double rx = xj[j] - px, ry = xj[nj + j] - py, rz = xj[2 * nj + j] - pz;
            const double ux = vj[j] - qx, uy = vj[nj + j] - qy, uz = vj[2 * nj + j] - qz;
            const double s = rx * rx + ry * ry + rz * rz + eps2;
            if (s == 0.0) continue;
            const double A = 1.0 / sqrt(s);
            const double B = A * A * A;
            const double C = B * A * A;
            const double ru = rx * ux + ry * uy + rz * uz;
            const double m = mj[j];
            ax += m * B * rx;
            ay += m * B * ry;
            az += m * B * rz;
            jx += m * (B * ux - 3.0 * C * ru * rx);
            jy += m * (B * uy - 3.0 * C * ru * ry);
            jz += m * (B * uz - 3.0 * C * ru * rz);
            ph -= m * A;
        }
        if (acc) { acc[i] = G * ax; acc[ni + i] = G * ay; acc[2 * ni + i] = G * az; }
        if (jerk) { jerk[i] = G * jx; jerk[ni + i] = G * jy; jerk[2 * ni + i] = G * jz; }
        if (pot) pot[i] = G * ph;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Adjoint of the force.  Given cotangents ga (3 x ni), gj (3 x ni, may be
 * NULL = 0) and gp (ni, may be NULL = 0) of the outputs above, returns the
 * cotangents of x_i, v_i (gxi, gvi), x_j, v_j (gxj, gvj) and m_j (gmj).
 * Any output may be NULL.
 *
 * Per pair (i <- j), with r, u, s, A, B, C as above and D = A^7, the pair's
 * share of  L = ga.a_i + gj.jerk_i + gp phi_i  is
 *   L_ij = G m_j [ B (ga.r) + B (gj.u) - 3 C (r.u)(gj.r) - gp A ]
 * and its derivatives (dA/dr = -B r, dB/dr = -3 C r, dC/dr = -5 D r) are
 *   g_r = G m_j [ B ga - 3C (ga.r) r - 3C (gj.u) r + 15 D (r.u)(gj.r) r
 *                 - 3C (gj.r) u - 3C (r.u) gj + gp B r ]
 *   g_u = G m_j [ B gj - 3C (gj.r) r ]
 *   dL_ij/dm_j = L_ij / m_j
 * Since r = x_j - x_i and u = v_j - v_i:  x_j gets +g_r, x_i gets -g_r,
 * v_j gets +g_u, v_i gets -g_u.  The same pairs as the forward are used
 * (self skipped by index; s == 0 skipped).
 * ---------------------------------------------------------------------- */
static void pair_adjoint(double rx, double ry, double rz, double ux, double uy, double uz,
                         double eps2, double m, double G,
                         const double ga[3], const double gj[3], double gp,
                         double gr[3], double gu[3], double *gm, int *skip) {
    const double s = rx * rx + ry * ry + rz * rz + eps2;
    if (s == 0.0) { *skip = 1; return; }
    *skip = 0;
    const double A = 1.0 / sqrt(s);
    const double B = A * A * A;
    const double C = B * A * A;
    const double D = C * A * A;
    const double ru = rx * ux + ry * uy + rz * uz;
    const double gar = ga[0] * rx + ga[1] * ry + ga[2] * rz;
    const double gjr = gj[0] * rx + gj[1] * ry + gj[2] * rz;
    const double gju = gj[0] * ux + gj[1] * uy + gj[2] * uz;
    const double r3[3] = {rx, ry, rz}, u3[3] = {ux, uy, uz};
    for (int k = 0; k < 3; ++k) {
        gr[k] = G * m * (B * ga[k] - 3.0 * C * gar * r3[k] - 3.0 * C * gju * r3[k]
                         + 15.0 * D * ru * gjr * r3[k] - 3.0 * C * gjr * u3[k]
                         - 3.0 * C * ru * gj[k] + gp * B * r3[k]);
        gu[k] = G * m * (B * gj[k] - 3.0 * C * gjr * r3[k]);
    }
    *gm = G * (B * gar + B * gju - 3.0 * C * ru * gjr - gp * A);
}

int oracle_force_vjp(int64_t ni, const double *xi, const double *vi, const int64_t *iself,
                     int64_t nj, const double *xj, const double *vj, const double *mj,
                     double G, double eps,
                     const double *ga, const double *gj, const double *gp,
                     double *gxi, double *gvi, double *gxj, double *gvj, double *gmj,
                     int nthreads) {
    if (ni < 0 || nj < 0 || eps < 0 || !ga) return -1;
    set_threads(nthreads);
    const double eps2 = eps * eps;
    int64_t i, j;
    /* i side: sum over j of -g_r, -g_u */
    if (gxi || gvi) {
#pragma omp parallel for schedule(static)
        for (i = 0; i < ni; ++i) {
            const double cga[3] = {ga[i], ga[ni + i], ga[2 * ni + i]};
            const double cgj[3] = {gj ? gj[i] : 0.0, gj ? gj[ni + i] : 0.0, gj ? gj[2 * ni + i] : 0.0};
            const double cgp = gp ? gp[i] : 0.0;
            const int64_t self = iself ? iself[i] : -1;
            double sx[3] = {0, 0, 0}, sv[3] = {0, 0, 0};
            for (int64_t jj = 0; jj < nj; ++jj) {
                if (jj == self) continue;
                double gr[3], gu[3], gm;
                int skip;
                pair_adjoint(xj[jj] - xi[i], xj[nj + jj] - xi[ni + i], xj[2 * nj + jj] - xi[2 * ni + i],
                             vj[jj] - vi[i], vj[nj + jj] - vi[ni + i], vj[2 * nj + jj] - vi[2 * ni + i],
                             eps2, mj[jj], G, cga, cgj, cgp, gr, gu, &gm, &skip);
                if (skip) continue;
                for (int k = 0; k < 3; ++k) { sx[k] -= gr[k]; sv[k] -= gu[k]; }
            }
            for (int k = 0; k < 3; ++k) {
                if (gxi) gxi[k * ni + i] = sx[k];
                if (gvi) gvi[k * ni + i] = sv[k];
            }
        }
    }
    /* j side: sum over i of +g_r, +g_u, dL/dm_j */
    if (gxj || gvj || gmj) {
#pragma omp parallel for schedule(static)
        for (j = 0; j < nj; ++j) {
            double sx[3] = {0, 0, 0}, sv[3] = {0, 0, 0}, sm = 0;
            for (int64_t ii = 0; ii < ni; ++ii) {
                if (iself && iself[ii] == j) continue;
                const double cga[3] = {ga[ii], ga[ni + ii], ga[2 * ni + ii]};
                const double cgj[3] = {gj ? gj[ii] : 0.0, gj ? gj[ni + ii] : 0.0, gj ? gj[2 * ni + ii] : 0.0};
                const double cgp = gp ? gp[ii] : 0.0;
                double gr[3], gu[3], gm;
                int skip;
                pair_adjoint(xj[j] - xi[ii], xj[nj + j] - xi[ni + ii], xj[2 * nj + j] - xi[2 * ni + ii],
                             vj[j] - vi[ii], vj[nj + j] - vi[ni + ii], vj[2 * nj + j] - vi[2 * ni + ii],
                             eps2, mj[j], G, cga, cgj, cgp, gr, gu, &gm, &skip);
                if (skip) continue;
                for (int k = 0; k < 3; ++k) { sx[k] += gr[k]; sv[k] += gu[k]; }
                sm += gm;
            }
            for (int k = 0; k < 3; ++k) {
                if (gxj) gxj[k * nj + j] = sx[k];
                if (gvj) gvj[k * nj + j] = sv[k];
            }
            if (gmj) gmj[j] = sm;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Hermite scheme (Makino & Aarseth 1992), one force evaluation per step.
 *
 * Predictor over Delta = t - t_0:
 *   x_p = x + v D + a D^2/2 + j D^3/6,   v_p = v + a D + j D^2/2
 * Corrector, with (a1, j1) evaluated at the predicted state:
 *   a2 = (-6 (a0 - a1) - D (4 j0 + 2 j1)) / D^2      (2nd derivative at t_0)
 *   a3 = (12 (a0 - a1) + 6 D (j0 + j1)) / D^3        (3rd derivative)
 *   x1 = x_p + a2 D^4/24 + a3 D^5/120
 *   v1 = v_p + a2 D^3/6  + a3 D^4/24
 * ---------------------------------------------------------------------- */
void oracle_predict_one(const double x[3], const double v[3], const double a[3],
                        const double j[3], double D, double xp[3], double vp[3]) {
    for (int k = 0; k < 3; ++k) {
        xp[k] = x[k] + v[k] * D + a[k] * D * D / 2.0 + j[k] * D * D * D / 6.0;
        vp[k] = v[k] + a[k] * D + j[k] * D * D / 2.0;
    }
}

void oracle_correct_one(const double xp[3], const double vp[3], const double a0[3],
                        const double j0[3], const double a1[3], const double j1[3], double D,
                        double x1[3], double v1[3], double a2[3], double a3[3]) {
    for (int k = 0; k < 3; ++k) {
        a2[k] = (-6.0 * (a0[k] - a1[k]) - D * (4.0 * j0[k] + 2.0 * j1[k])) / (D * D);
        a3[k] = (12.0 * (a0[k] - a1[k]) + 6.0 * D * (j0[k] + j1[k])) / (D * D * D);
        x1[k] = xp[k] + a2[k] * D * D * D * D / 24.0 + a3[k] * D * D * D * D * D / 120.0;
        v1[k] = vp[k] + a2[k] * D * D * D / 6.0 + a3[k] * D * D * D * D / 24.0;
    }
}

static double norm3(const double w[3]) { return sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]); }

/* Aarseth criterion at the end of a step:
 *   dt = sqrt(eta (|a1| |a2_1| + |j1|^2) / (|j1| |a3| + |a2_1|^2)),
 *   a2_1 = a2 + a3 D (second derivative carried to the new time). */
double oracle_aarseth_dt(const double a1[3], const double j1[3], const double a2[3],
                         const double a3[3], double D, double eta) {
    double a21[3];
    for (int k = 0; k < 3; ++k) a21[k] = a2[k] + a3[k] * D;
    const double na = norm3(a1), nj = norm3(j1), n2 = norm3(a21), n3 = norm3(a3);
    return sqrt(eta * (na * n2 + nj * nj) / (nj * n3 + n2 * n2));
}

/* Power-of-two time-step level in ticks.
 *  - q = largest 2^k with 2^k <= crit (time units), clamped to
 *    [2^lmin, 2^lmax]; a criterion that is zero, negative or not finite
 *    gives 2^lmin.
 *  - dt_old <= 0 means "first step": return q.
 *  - q < dt_old: return q (halving any number of times keeps t_new a
 *    multiple of the step).
 *  - q >= dt_old: the step may double once, and only if t_new is a
 *    multiple of 2 dt_old (and 2 dt_old <= 2^lmax); else it stays. */
int64_t oracle_quantise_dt(double crit, int64_t dt_old, int64_t t_new, int lmin, int lmax) {
    const int64_t dmin = (int64_t)1 << (lmin + 20), dmax = (int64_t)1 << (lmax + 20);
    int64_t q;
    if (!(crit > 0.0) || !isfinite(crit)) {
        q = dmin;
    } else {
        q = dmin;
        while (q < dmax && (double)(q * 2) * TICK <= crit) q *= 2;
    }
    if (dt_old <= 0) return q;
    if (q < dt_old) return q;
    if (q > dt_old && 2 * dt_old <= dmax && t_new % (2 * dt_old) == 0) return 2 * dt_old;
    return dt_old;
}

/* Active block: t_next = min_i (t_i + dt_i); active = all i with
 * t_i + dt_i == t_next, in ascending index order. */
int64_t oracle_select_active(int64_t n, const int64_t *t, const int64_t *dt,
                             int32_t *idx, int64_t *t_next_out) {
    if (n <= 0) return 0;
    int64_t tn = t[0] + dt[0];
    for (int64_t i = 1; i < n; ++i)
        if (t[i] + dt[i] < tn) tn = t[i] + dt[i];
    int64_t c = 0;
    for (int64_t i = 0; i < n; ++i)
        if (t[i] + dt[i] == tn) idx[c++] = (int32_t)i;
    if (t_next_out) *t_next_out = tn;
    return c;
}

/* ------------------------------------------------------------------------
 * Hermite integration driver.
 *
 * State (all n particles): x, v, a, j (3 x n each), m (n), t and dt (ticks).
 * opts: G, eps, eta, eta_s; levels [lmin, lmax] (log2 of time units);
 * shared_log2 != 0 selects one shared step 2^shared_log2 for every particle.
 *
 * init != 0: compute a, j at the given x, v (all particles, self excluded)
 * and the first steps dt = q(eta_s |a| / |j|) (shared mode: 2^shared_log2);
 * t is left as given (normally 0).
 *
 * Then block steps are taken until every t_i == t_end (t_end must be a
 * multiple of the largest step for that to happen exactly; the loop stops
 * at the first block time beyond t_end otherwise).  One block step:
 *   1. select the active block and t_next;
 *   2. predict every particle to t_next from its own t_j;
 *   3. evaluate a1, j1 for the active particles at their predicted state
 *      against all predicted particles (self excluded);
 *   4. correct the active particles over D = dt_i, store a1, j1, t_i = t_next;
 *   5. new dt_i by the Aarseth criterion and oracle_quantise_dt
 *      (shared mode: unchanged).
 * Returns the number of block steps; *sum_active accumulates sum N_act.
 * ---------------------------------------------------------------------- */
typedef struct {
    double G, eps, eta, eta_s;
    int lmin, lmax, shared_log2;
} oracle_hermite_opts;

static int64_t first_dt(const oracle_hermite_opts *o, const double a[3], const double j[3]) {
    if (o->shared_log2 != 0) return (int64_t)1 << (o->shared_log2 + 20);
    const double na = norm3(a), nj = norm3(j);
    return oracle_quantise_dt(o->eta_s * na / nj, 0, 0, o->lmin, o->lmax);
}

int64_t oracle_hermite_run(int64_t n, double *x, double *v, double *a, double *jk,
                           const double *m, int64_t *t, int64_t *dt,
                           const oracle_hermite_opts *o, int init, int64_t t_end,
                           int64_t max_steps, int64_t *sum_active, int nthreads) {
    int64_t *self = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    double *xp = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *vp = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *xa = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *va = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *a1 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *j1 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *aself = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    if (!self || !xp || !vp || !xa || !va || !a1 || !j1 || !idx || !aself) {
        free(self); free(xp); free(vp); free(xa); free(va); free(a1); free(j1); free(idx); free(aself);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) self[i] = i;
    if (init) {
        oracle_force(n, x, v, self, n, x, v, m, o->G, o->eps, a, jk, NULL, nthreads);
        for (int64_t i = 0; i < n; ++i) {
            const double ai[3] = {a[i], a[n + i], a[2 * n + i]};
            const double ji[3] = {jk[i], jk[n + i], jk[2 * n + i]};
            dt[i] = first_dt(o, ai, ji);
        }
    }
    int64_t steps = 0;
    while (steps < max_steps) {
        int64_t tn;
        const int64_t na = oracle_select_active(n, t, dt, idx, &tn);
        if (na == 0 || tn > t_end) break;
        /* 2. predict all */
        for (int64_t i = 0; i < n; ++i) {
            const double D = (double)(tn - t[i]) * TICK;
            const double xi[3] = {x[i], x[n + i], x[2 * n + i]}, vi[3] = {v[i], v[n + i], v[2 * n + i]};
            const double ai[3] = {a[i], a[n + i], a[2 * n + i]}, ji[3] = {jk[i], jk[n + i], jk[2 * n + i]};
            double xo[3], vo[3];
            oracle_predict_one(xi, vi, ai, ji, D, xo, vo);
            for (int k = 0; k < 3; ++k) { xp[k * n + i] = xo[k]; vp[k * n + i] = vo[k]; }
        }
        /* 3. forces on the active block */
        for (int64_t c = 0; c < na; ++c) {
            const int64_t i = idx[c];
            for (int k = 0; k < 3; ++k) { xa[k * na + c] = xp[k * n + i]; va[k * na + c] = vp[k * n + i]; }
            aself[c] = i;
        }
        oracle_force(na, xa, va, aself, n, xp, vp, m, o->G, o->eps, a1, j1, NULL, nthreads);
        /* 4-5. correct and choose new steps */
        for (int64_t c = 0; c < na; ++c) {
            const int64_t i = idx[c];
            const double D = (double)dt[i] * TICK;
            double xo[3], vo[3], a0[3], j0[3], an[3], jn[3], x1[3], v1[3], a2[3], a3[3];
            for (int k = 0; k < 3; ++k) {
                xo[k] = xp[k * n + i]; vo[k] = vp[k * n + i];
                a0[k] = a[k * n + i]; j0[k] = jk[k * n + i];
                an[k] = a1[k * na + c]; jn[k] = j1[k * na + c];
            }
            oracle_correct_one(xo, vo, a0, j0, an, jn, D, x1, v1, a2, a3);
            for (int k = 0; k < 3; ++k) {
                x[k * n + i] = x1[k]; v[k * n + i] = v1[k];
                a[k * n + i] = an[k]; jk[k * n + i] = jn[k];
            }
            t[i] = tn;
            if (o->shared_log2 == 0) {
                const double crit = oracle_aarseth_dt(an, jn, a2, a3, D, o->eta);
                dt[i] = oracle_quantise_dt(crit, dt[i], tn, o->lmin, o->lmax);
            }
        }
        ++steps;
        if (sum_active) *sum_active += na;
    }
    free(self); free(xp); free(vp); free(xa); free(va); free(a1); free(j1); free(idx); free(aself);
    return steps;
}

/* Energy at a common time: E_kin = sum m v^2 / 2, E_pot = sum m phi / 2,
 * phi with self excluded (Eq. 2 uses E = E_kin + E_pot). */
int oracle_energy(int64_t n, const double *x, const double *v, const double *m,
                  double G, double eps, double *ekin, double *epot, int nthreads) {
    int64_t *self = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    double *phi = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!self || !phi) { free(self); free(phi); return -1; }
    for (int64_t i = 0; i < n; ++i) self[i] = i;
    oracle_force(n, x, v, self, n, x, v, m, G, eps, NULL, NULL, phi, nthreads);
    double k = 0, p = 0;
    for (int64_t i = 0; i < n; ++i) {
        k += 0.5 * m[i] * (v[i] * v[i] + v[n + i] * v[n + i] + v[2 * n + i] * v[2 * n + i]);
        p += 0.5 * m[i] * phi[i];
    }
    *ekin = k;
    *epot = p;
    free(self); free(phi);
    return 0;
}

/* ------------------------------------------------------------------------
 * Shared-step Hermite run and its adjoint (all particles active, step
 * D = dt for nsteps steps, starting from x0, v0 with a0, j0 evaluated at
 * the start).  Used to differentiate L(x(T)) with respect to x0, v0, m.
 *
 * Forward step (state x, v, a, j -> x1, v1, a1, j1):
 *   predictor (above) -> (a1, j1) = F(x_p, v_p, m) -> corrector (above).
 * Backward step, for state cotangents (X, V, Aa, Jj) of the new state:
 *   P2 = X D^4/24 + V D^3/6,   P3 = X D^5/120 + V D^4/24       (on a2, a3)
 *   force cotangents: ga = Aa + 6 P2/D^2 - 12 P3/D^3,
 *                     gj = Jj - 2 P2/D + 6 P3/D^2
 *   (gx_p, gv_p, gm) = (X, V, 0) + VJP of F at (x_p, v_p) for (ga, gj)
 *   old state: X' = gx_p,  V' = D gx_p + gv_p,
 *              Aa' = -6 P2/D^2 + 12 P3/D^3 + D^2/2 gx_p + D gv_p,
 *              Jj' = -4 P2/D + 6 P3/D^2 + D^3/6 gx_p + D^2/2 gv_p.
 * At the start (a0, j0) = F(x0, v0): the final (Aa, Jj) go through one
 * more VJP into gx0, gv0, gm.
 * ---------------------------------------------------------------------- */
int oracle_hermite_shared_forward(int64_t n, double *x, double *v, const double *m,
                                  double G, double eps, double D, int64_t nsteps,
                                  double *xp_hist, double *vp_hist, int nthreads) {
    int64_t *self = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double *a = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *jk = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *a1 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *j1 = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *xp = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *vp = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!self || !a || !jk || !a1 || !j1 || !xp || !vp) {
        free(self); free(a); free(jk); free(a1); free(j1); free(xp); free(vp);
        return -1;
    }
    for (int64_t i = 0; i < n; ++i) self[i] = i;
    oracle_force(n, x, v, self, n, x, v, m, G, eps, a, jk, NULL, nthreads);
    for (int64_t s = 0; s < nsteps; ++s) {
        for (int64_t i = 0; i < n; ++i) {
            double xi[3], vi[3], ai[3], ji[3], xo[3], vo[3];
            for (int k = 0; k < 3; ++k) { xi[k] = x[k * n + i]; vi[k] = v[k * n + i]; ai[k] = a[k * n + i]; ji[k] = jk[k * n + i]; }
            oracle_predict_one(xi, vi, ai, ji, D, xo, vo);
            for (int k = 0; k < 3; ++k) { xp[k * n + i] = xo[k]; vp[k * n + i] = vo[k]; }
        }
        if (xp_hist) memcpy(xp_hist + (size_t)s * 3 * n, xp, sizeof(double) * 3 * (size_t)n);
        if (vp_hist) memcpy(vp_hist + (size_t)s * 3 * n, vp, sizeof(double) * 3 * (size_t)n);
        oracle_force(n, xp, vp, self, n, xp, vp, m, G, eps, a1, j1, NULL, nthreads);
        for (int64_t i = 0; i < n; ++i) {
            double xo[3], vo[3], a0[3], j0[3], an[3], jn[3], x1[3], v1[3], a2[3], a3[3];
            for (int k = 0; k < 3; ++k) {
                xo[k] = xp[k * n + i]; vo[k] = vp[k * n + i]; a0[k] = a[k * n + i]; j0[k] = jk[k * n + i];
                an[k] = a1[k * n + i]; jn[k] = j1[k * n + i];
            }
            oracle_correct_one(xo, vo, a0, j0, an, jn, D, x1, v1, a2, a3);
            for (int k = 0; k < 3; ++k) { x[k * n + i] = x1[k]; v[k * n + i] = v1[k]; a[k * n + i] = an[k]; jk[k * n + i] = jn[k]; }
        }
    }
    free(self); free(a); free(jk); free(a1); free(j1); free(xp); free(vp);
    return 0;
}

int oracle_hermite_shared_adjoint(int64_t n, const double *x0, const double *v0, const double *m,
                                  double G, double eps, double D, int64_t nsteps,
                                  const double *gx_end, const double *gv_end,
                                  double *gx0, double *gv0, double *gm, int nthreads) {
    const size_t s3 = 3 * (size_t)n;
    double *xp_hist = (double *)malloc(sizeof(double) * s3 * (size_t)(nsteps > 0 ? nsteps : 1));
    double *vp_hist = (double *)malloc(sizeof(double) * s3 * (size_t)(nsteps > 0 ? nsteps : 1));
    double *x = (double *)malloc(sizeof(double) * s3), *v = (double *)malloc(sizeof(double) * s3);
    double *X = (double *)malloc(sizeof(double) * s3), *V = (double *)malloc(sizeof(double) * s3);
    double *Aa = (double *)calloc(s3, sizeof(double)), *Jj = (double *)calloc(s3, sizeof(double));
    double *ga = (double *)malloc(sizeof(double) * s3), *gj = (double *)malloc(sizeof(double) * s3);
    double *tx = (double *)malloc(sizeof(double) * s3), *tv = (double *)malloc(sizeof(double) * s3);
    double *tm = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t *self = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int rc = 0;
    if (!xp_hist || !vp_hist || !x || !v || !X || !V || !Aa || !Jj || !ga || !gj || !tx || !tv || !tm || !self) {
        rc = -1;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) self[i] = i;
    memcpy(x, x0, sizeof(double) * s3);
    memcpy(v, v0, sizeof(double) * s3);
    oracle_hermite_shared_forward(n, x, v, m, G, eps, D, nsteps, xp_hist, vp_hist, nthreads);
    memcpy(X, gx_end, sizeof(double) * s3);
    if (gv_end) memcpy(V, gv_end, sizeof(double) * s3); else memset(V, 0, sizeof(double) * s3);
    for (int64_t i = 0; i < n; ++i) gm[i] = 0.0;
    for (int64_t s = nsteps - 1; s >= 0; --s) {
        const double *xp = xp_hist + (size_t)s * s3, *vp = vp_hist + (size_t)s * s3;
        for (size_t q = 0; q < s3; ++q) {
            const double P2 = X[q] * D * D * D * D / 24.0 + V[q] * D * D * D / 6.0;
            const double P3 = X[q] * D * D * D * D * D / 120.0 + V[q] * D * D * D * D / 24.0;
            ga[q] = Aa[q] + 6.0 * P2 / (D * D) - 12.0 * P3 / (D * D * D);
            gj[q] = Jj[q] - 2.0 * P2 / D + 6.0 * P3 / (D * D);
            Aa[q] = -6.0 * P2 / (D * D) + 12.0 * P3 / (D * D * D);
            Jj[q] = -4.0 * P2 / D + 6.0 * P3 / (D * D);
        }
        oracle_force_vjp(n, xp, vp, self, n, xp, vp, m, G, eps, ga, gj, NULL,
                         tx, tv, NULL, NULL, NULL, nthreads);
        /* The fused i == j adjoint: add the j-side half as well. */
        {
            double *ux = (double *)malloc(sizeof(double) * s3), *uv = (double *)malloc(sizeof(double) * s3);
            double *um = (double *)malloc(sizeof(double) * (size_t)n);
            if (!ux || !uv || !um) { free(ux); free(uv); free(um); rc = -1; goto done; }
            oracle_force_vjp(n, xp, vp, self, n, xp, vp, m, G, eps, ga, gj, NULL,
                             NULL, NULL, ux, uv, um, nthreads);
            for (size_t q = 0; q < s3; ++q) { tx[q] += ux[q]; tv[q] += uv[q]; }
            for (int64_t i = 0; i < n; ++i) gm[i] += um[i];
            free(ux); free(uv); free(um);
        }
        for (size_t q = 0; q < s3; ++q) {
            const double gxp = X[q] + tx[q], gvp = V[q] + tv[q];
            X[q] = gxp;
            V[q] = D * gxp + gvp;
            Aa[q] += D * D / 2.0 * gxp + D * gvp;
            Jj[q] += D * D * D / 6.0 * gxp + D * D / 2.0 * gvp;
        }
    }
    /* initial evaluation (a0, j0) = F(x0, v0) */
    {
        double *ux = (double *)malloc(sizeof(double) * s3), *uv = (double *)malloc(sizeof(double) * s3);
        double *um = (double *)malloc(sizeof(double) * (size_t)n);
        if (!ux || !uv || !um) { free(ux); free(uv); free(um); rc = -1; goto done; }
        oracle_force_vjp(n, x0, v0, self, n, x0, v0, m, G, eps, Aa, Jj, NULL,
                         tx, tv, ux, uv, um, nthreads);
        for (size_t q = 0; q < s3; ++q) { gx0[q] = X[q] + tx[q] + ux[q]; gv0[q] = V[q] + tv[q] + uv[q]; }
        for (int64_t i = 0; i < n; ++i) gm[i] += um[i];
        free(ux); free(uv); free(um);
    }
done:
    free(xp_hist); free(vp_hist); free(x); free(v); free(X); free(V); free(Aa); free(Jj);
    free(ga); free(gj); free(tx); free(tv); free(tm); free(self);
    return rc;
}

/* ------------------------------------------------------------------------
 * Nearest neighbour (Section 3.3: besides force, jerk and potential the
 * GRAPE reports, for every i-particle being updated, the particle closest
 * to it; the GPU finds it with one distance comparison per pair inside the
 * force loop).
 *
 * For each i: nn[i] is the j != iself[i] with the smallest unsoftened
 * squared distance |x_j - x_i|^2, the lowest such j when several are equally
 * close; r2[i] is that squared distance.  With no candidate (nj == 0, or
 * the only j is i itself) nn[i] = -1 and r2[i] = +inf.  Coincident
 * distinct particles are candidates at distance 0.
 * ---------------------------------------------------------------------- */
int oracle_nearest(int64_t ni, const double *xi, const int64_t *iself, int64_t nj, const double *xj,
                   int64_t *nn, double *r2, int nthreads) {
    if (ni < 0 || nj < 0) return -1;
    set_threads(nthreads);
    int64_t i;
#pragma omp parallel for schedule(static)
    for (i = 0; i < ni; ++i) {
        const double px = xi[i], py = xi[ni + i], pz = xi[2 * ni + i];
        const int64_t self = iself ? iself[i] : -1;
        int64_t best = -1;
        double bd = INFINITY;
        for (int64_t j = 0; j < nj; ++j) {
            if (j == self) continue;
            const double rx = xj[j] - px, ry = xj[nj + j] - py, rz = xj[2 * nj + j] - pz;
            const double d = rx * rx + ry * ry + rz * rz;
            if (d < bd) {   /* strict: the first (lowest) j wins a tie */
                bd = d;
                best = j;
            }
        }
        nn[i] = best;
        r2[i] = bd;
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Shared-step leapfrog driven by acceleration alone.  Section 4 runs a
 * Barnes-Hut treecode on the library with the jerk and nearest-neighbour
 * work switched off, since such integrators need only the acceleration;
 * the standard second-order kick-drift-kick (velocity Verlet) form of one
 * step of length dt is
 *   v_h = v_0 + a_0 dt/2,   x_1 = x_0 + v_h dt,
 *   a_1 = a(x_1),           v_1 = v_h + a_1 dt/2,
 * with a(x) the softened acceleration of every particle from all others
 * (self excluded by index).  acc holds a(x) on entry when have_acc != 0
 * (else it is computed first) and a(x) at the end on return; pot (may be
 * NULL) receives the potential at the end.  x, v, acc are 3 x n rows and
 * are updated in place.
 * ---------------------------------------------------------------------- */
int oracle_leapfrog(int64_t n, double *x, double *v, const double *m, double G, double eps, double dt,
                    int64_t nsteps, double *acc, double *pot, int have_acc, int nthreads) {
    if (n < 0 || nsteps < 0 || eps < 0) return -1;
    if (n == 0) return 0;
    int64_t *self = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    double *ph = (double *)malloc(sizeof(double) * (size_t)n);
    if (!self || !ph) {
        free(self);
        free(ph);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i) self[i] = i;
    int rc = 0;
    if (!have_acc) rc = oracle_force(n, x, v, self, n, x, v, m, G, eps, acc, NULL, ph, nthreads);
    const double h = 0.5 * dt;
    for (int64_t s = 0; s < nsteps && rc == 0; ++s) {
        for (int64_t k = 0; k < 3 * n; ++k) {
            v[k] += acc[k] * h;
            x[k] += v[k] * dt;
        }
        rc = oracle_force(n, x, v, self, n, x, v, m, G, eps, acc, NULL, ph, nthreads);
        for (int64_t k = 0; k < 3 * n; ++k) v[k] += acc[k] * h;
    }
    if (rc == 0 && pot) {
        if (nsteps == 0 && have_acc) rc = oracle_force(n, x, v, self, n, x, v, m, G, eps, NULL, NULL, ph, nthreads);
        memcpy(pot, ph, sizeof(double) * (size_t)n);
    }
    free(self);
    free(ph);
    return rc;
}
