/*
 * hermite_oracle.c -- CPU reference for the fewbody integrator.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, FP64 implementation of
 * the fourth-order time-symmetrised Hermite predictor-corrector (Kokubo et
 * al. 1998, as used in Section 2.2.1 and Algorithm 2 of the Swarm-NG paper,
 * arXiv:1208.1157), iterated P(EC)^n over independent few-body systems.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header, table or helper with the HIP
 * library, and the HIP library never calls it.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no SIMD intrinsics, no
 * fused multiply-add), so every operation below rounds exactly as written.
 *
 * Layout: one system at a time; body b, component c at index 3*b + c.
 * Body 0 is the central star.  G = 1 (Section 2.1).
 *
 * Readings of the paper used here (the paper's text is garbled or silent):
 *  - Eq. 4 corrector: coefficient 3/20 (printed 3/10), jerk term multiplies
 *    (dt)^3 (Algorithm 2 prints dt), and both the x and v updates start from
 *    the predicted state of the current step at every iteration.
 *  - Two acceleration/jerk evaluations per step (P(EC)^2); the step's last
 *    evaluation becomes a0, j0 of the next step; the first a0, j0 come from
 *    one evaluation at set-up (the "prepare" call of Algorithm 1).
 *  - Eq. 6 energy: the potential sums each pair once (i < j).
 *  - Angular momentum about the origin: L = sum m x cross v.
 *  - Adaptive step (not the paper's Eq. 5): dt = eta * min over pairs of
 *    |a_ij| / |j_ij| for the pairwise two-body acceleration and jerk, taken
 *    from the step's last evaluation state; the last step is clamped to
 *    land on t_end.
 *  - Stop rules: planet-planet separation below one mutual Hill radius
 *    ((m_i+m_j)/(3 m0))^(1/3) (r_i+r_j)/2 with r the astrocentric distance;
 *    any planet farther than r_eject from the star; non-finite state.
 */
#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#define ORA_MAX_BODIES 512

/* status codes (same meaning as the library's, defined independently) */
enum {
    ORA_ACTIVE = 0, ORA_DONE = 1, ORA_ENCOUNTER = 2, ORA_EJECTED = 3,
    ORA_NONFINITE = 4, ORA_STALLED_DT = 5, ORA_MAXSTEPS = 6
};

/* ------------------------------------------------------------------------ */
/* Eq. 1 and its time derivative.                                            */
/* For a pair (i, j) with r = x_j - x_i and u = v_j - v_i the acceleration   */
/* per unit mass is A = r / |r|^3 and the jerk per unit mass is              */
/* J = u / |r|^3 - 3 (r.u) r / |r|^5.  Body i gains +m_j A, body j gains     */
/* -m_i A (Newton's third law), and likewise for J.  Pairs are visited with  */
/* planet-planet pairs first and the star's pairs last (Section 4.2), each   */
/* group in lexicographic (i < j) order.                                     */
/* ------------------------------------------------------------------------ */
static void pair_accumulate(int i, int j, const double *m, const double *x,
                            const double *v, double *a, double *jk)
{
    double r[3], u[3], A[3], J[3];
    for (int c = 0; c < 3; ++c) {
        r[c] = x[3 * j + c] - x[3 * i + c];
        u[c] = v[3 * j + c] - v[3 * i + c];
    }
    double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double ru = r[0] * u[0] + r[1] * u[1] + r[2] * u[2];
    double s = 1.0 / sqrt(r2);
    double s2 = s * s;
    double s3 = s2 * s;
    for (int c = 0; c < 3; ++c) {
        A[c] = r[c] * s3;
        J[c] = u[c] * s3 - 3.0 * ru * s2 * A[c];
    }
    for (int c = 0; c < 3; ++c) {
        a[3 * i + c] = a[3 * i + c] + m[j] * A[c];
        a[3 * j + c] = a[3 * j + c] - m[i] * A[c];
        jk[3 * i + c] = jk[3 * i + c] + m[j] * J[c];
        jk[3 * j + c] = jk[3 * j + c] - m[i] * J[c];
    }
}

void ora_accjerk(int n, const double *m, const double *x, const double *v,
                 double *a, double *jk)
{
    for (int k = 0; k < 3 * n; ++k) {
        a[k] = 0.0;
        jk[k] = 0.0;
    }
    for (int i = 1; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            pair_accumulate(i, j, m, x, v, a, jk);
    for (int j = 1; j < n; ++j)
        pair_accumulate(0, j, m, x, v, a, jk);
}

/* Eq. 3: Taylor predictor to the jerk. */
void ora_predict(int n, double h, const double *x0, const double *v0,
                 const double *a0, const double *j0, double *xp, double *vp)
{
    double h2 = h * h, h3 = h2 * h;
    for (int k = 0; k < 3 * n; ++k) {
        xp[k] = x0[k] + v0[k] * h + 0.5 * a0[k] * h2 + j0[k] * h3 / 6.0;
        vp[k] = v0[k] + a0[k] * h + 0.5 * j0[k] * h2;
    }
}

/* Eq. 4 (as read above): correction from the predicted state (xp, vp)
 * using the start-of-step (a0, j0) and the latest evaluation (ak, jk). */
void ora_correct(int n, double h, const double *xp, const double *vp,
                 const double *a0, const double *j0, const double *ak,
                 const double *jk, double *xc, double *vc)
{
    double h2 = h * h, h3 = h2 * h;
    for (int k = 0; k < 3 * n; ++k) {
        xc[k] = xp[k] - (3.0 / 20.0) * (a0[k] - ak[k]) * h2
                      - (7.0 * j0[k] + 2.0 * jk[k]) * h3 / 60.0;
        vc[k] = vp[k] - 0.5 * (a0[k] - ak[k]) * h
                      - (5.0 * j0[k] + jk[k]) * h2 / 12.0;
    }
}

/* One Hermite step (Algorithm 2).  x, v, a0, j0 are updated in place.
 * n_corr evaluation+correction passes (2 = P(EC)^2).  If converged != 0 the
 * corrector is iterated until (x, v) stop changing bitwise (at most 50
 * passes), which gives the time-symmetric limit of the scheme. */
static void hermite_step(int n, const double *m, double *x, double *v,
                         double *a0, double *j0, double h, int n_corr,
                         int converged)
{
    double xp[3 * ORA_MAX_BODIES], vp[3 * ORA_MAX_BODIES];
    double xc[3 * ORA_MAX_BODIES], vc[3 * ORA_MAX_BODIES];
    double xn[3 * ORA_MAX_BODIES], vn[3 * ORA_MAX_BODIES];
    double ak[3 * ORA_MAX_BODIES], jk[3 * ORA_MAX_BODIES];
    ora_predict(n, h, x, v, a0, j0, xp, vp);
    memcpy(xc, xp, sizeof(double) * 3 * n);
    memcpy(vc, vp, sizeof(double) * 3 * n);
    int passes = converged ? 50 : n_corr;
    for (int it = 0; it < passes; ++it) {
        ora_accjerk(n, m, xc, vc, ak, jk);
        ora_correct(n, h, xp, vp, a0, j0, ak, jk, xn, vn);
        int same = memcmp(xn, xc, sizeof(double) * 3 * n) == 0 &&
                   memcmp(vn, vc, sizeof(double) * 3 * n) == 0;
        memcpy(xc, xn, sizeof(double) * 3 * n);
        memcpy(vc, vn, sizeof(double) * 3 * n);
        if (converged && same)
            break;
    }
    memcpy(x, xc, sizeof(double) * 3 * n);
    memcpy(v, vc, sizeof(double) * 3 * n);
    if (converged) {
        ora_accjerk(n, m, x, v, a0, j0);
    } else {
        memcpy(a0, ak, sizeof(double) * 3 * n);
        memcpy(j0, jk, sizeof(double) * 3 * n);
    }
}

/* Fixed-step integration of one system for nsteps steps of size h.
 * flags bit 0: compute (a0, j0) from (x, v) first (set-up evaluation).
 * flags bit 1: converged (time-symmetric) corrector, test use only.
 * Returns 0, or -1 for bad arguments. */
int ora_integrate_fixed(int n, const double *m, double *x, double *v,
                        double *a0, double *j0, double h, long nsteps,
                        int n_corr, int flags)
{
    if (n < 1 || n > ORA_MAX_BODIES || n_corr < 1 || nsteps < 0)
        return -1;
    if (flags & 1)
        ora_accjerk(n, m, x, v, a0, j0);
    for (long k = 0; k < nsteps; ++k)
        hermite_step(n, m, x, v, a0, j0, h, n_corr, (flags & 2) != 0);
    return 0;
}

/* Eq. 6 with each pair counted once; angular momentum about the origin. */
void ora_energy(int n, const double *m, const double *x, const double *v,
                double *energy, double *angmom)
{
    double kin = 0.0, pot = 0.0;
    double L[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < n; ++i) {
        const double *xi = x + 3 * i, *vi = v + 3 * i;
        kin = kin + 0.5 * m[i] * (vi[0] * vi[0] + vi[1] * vi[1] + vi[2] * vi[2]);
        L[0] = L[0] + m[i] * (xi[1] * vi[2] - xi[2] * vi[1]);
        L[1] = L[1] + m[i] * (xi[2] * vi[0] - xi[0] * vi[2]);
        L[2] = L[2] + m[i] * (xi[0] * vi[1] - xi[1] * vi[0]);
    }
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double d[3];
            for (int c = 0; c < 3; ++c)
                d[c] = x[3 * i + c] - x[3 * j + c];
            pot = pot + m[i] * m[j] / sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        }
    *energy = kin - pot;
    angmom[0] = L[0];
    angmom[1] = L[1];
    angmom[2] = L[2];
}

/* ------------------------------------------------------------------------ */
/* Adaptive step and stop rules (readings listed in the header).             */
/* ------------------------------------------------------------------------ */

/* eta * min over pairs of |a_ij| / |j_ij| where a_ij = (m_i+m_j) r/|r|^3 is
 * the pair's relative two-body acceleration and j_ij its time derivative.
 * Both are formed explicitly here; the mass factor cancels in the ratio. */
double ora_pair_timestep(int n, const double *m, const double *x,
                         const double *v, double eta)
{
    double best = INFINITY;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double r[3], u[3], A[3], J[3];
            for (int c = 0; c < 3; ++c) {
                r[c] = x[3 * j + c] - x[3 * i + c];
                u[c] = v[3 * j + c] - v[3 * i + c];
            }
            double mu = m[i] + m[j];
            double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
            double rn = sqrt(r2);
            double ru = r[0] * u[0] + r[1] * u[1] + r[2] * u[2];
            for (int c = 0; c < 3; ++c) {
                A[c] = mu * r[c] / (r2 * rn);
                J[c] = mu * (u[c] / (r2 * rn) - 3.0 * ru * r[c] / (r2 * r2 * rn));
            }
            double na = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
            double nj = sqrt(J[0] * J[0] + J[1] * J[1] + J[2] * J[2]);
            double q = na / nj;
            if (q < best)
                best = q;
        }
    return eta * best;
}

/* Eq. 5 (Section 4.3.1): dt = tau [sum_i |j_i|^2 / |a_i|^2]^(-1/2) over the
 * bodies, from the acceleration and jerk at the beginning of the step. */
double ora_paper_timestep(int n, const double *a0, const double *j0, double tau)
{
    double sum = 0.0;
    for (int i = 0; i < n; ++i) {
        const double *a = a0 + 3 * i, *j = j0 + 3 * i;
        double aa = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
        double jj = j[0] * j[0] + j[1] * j[1] + j[2] * j[2];
        sum = sum + jj / aa;
    }
    return tau / sqrt(sum);
}

/* Status after a committed step, from the stop rules.  stop_rules bit 0
 * enables the close-encounter test, bit 1 the ejection test. */
int ora_check_stop(int n, const double *m, const double *x, const double *v,
                   int stop_rules, double r_eject)
{
    for (int k = 0; k < 3 * n; ++k)
        if (!isfinite(x[k]) || !isfinite(v[k]))
            return ORA_NONFINITE;
    double rs[ORA_MAX_BODIES];
    for (int i = 1; i < n; ++i) {
        double d[3];
        for (int c = 0; c < 3; ++c)
            d[c] = x[3 * i + c] - x[c];
        rs[i] = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    }
    if (stop_rules & 1) {
        for (int i = 1; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                double d[3];
                for (int c = 0; c < 3; ++c)
                    d[c] = x[3 * i + c] - x[3 * j + c];
                double sep = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
                double hill = cbrt((m[i] + m[j]) / (3.0 * m[0])) * 0.5 * (rs[i] + rs[j]);
                if (sep < hill)
                    return ORA_ENCOUNTER;
            }
    }
    if (stop_rules & 2) {
        for (int i = 1; i < n; ++i)
            if (rs[i] > r_eject)
                return ORA_EJECTED;
    }
    return ORA_ACTIVE;
}

/* Adaptive integration of one system from *t to t_end.
 * Algorithm 1's loop: while active and steps < max_steps, advance, then
 * check.  The step size of each step is the one the previous step's last
 * evaluation proposed (*dt_next; the set-up evaluation proposes the first
 * one).  A step that would pass t_end is shortened to end on it and sets t
 * to t_end exactly.  A proposed step below 1e-12 |t_end| stalls the system.
 * flags bit 0: set-up evaluation of (a0, j0) and *dt_next first.
 * flags bit 1: Eq. 5's rule (eta is tau; dt from the step's starting a0, j0,
 * which are the previous step's last evaluation) instead of the pairwise
 * rule.
 * Returns the final status. */
int ora_integrate_adaptive(int n, const double *m, double *x, double *v,
                           double *a0, double *j0, double *t, double t_end,
                           double eta, int stop_rules, double r_eject,
                           long max_steps, double *dt_next, long *steps,
                           int flags)
{
    if (n < 2 || n > ORA_MAX_BODIES)
        return -1;
    const int paper_rule = (flags & 2) != 0;
    if (flags & 1) {
        ora_accjerk(n, m, x, v, a0, j0);
        *dt_next = paper_rule ? ora_paper_timestep(n, a0, j0, eta)
                              : ora_pair_timestep(n, m, x, v, eta);
    }
    double xp[3 * ORA_MAX_BODIES], vp[3 * ORA_MAX_BODIES];
    double xc[3 * ORA_MAX_BODIES], vc[3 * ORA_MAX_BODIES];
    double ak[3 * ORA_MAX_BODIES], jk[3 * ORA_MAX_BODIES];
    int status = ORA_ACTIVE;
    while (status == ORA_ACTIVE) {
        if (*t >= t_end) {
            status = ORA_DONE;
            break;
        }
        if (*steps >= max_steps) {
            status = ORA_MAXSTEPS;
            break;
        }
        if (isnan(*dt_next)) {
            status = ORA_NONFINITE;
            break;
        }
        if (!(*dt_next >= 1e-12 * fabs(t_end))) {
            status = ORA_STALLED_DT;
            break;
        }
        int last = *t + *dt_next >= t_end;
        double h = last ? t_end - *t : *dt_next;
        /* one P(EC)^2 step; remember the state of the last evaluation */
        ora_predict(n, h, x, v, a0, j0, xp, vp);
        memcpy(xc, xp, sizeof(double) * 3 * n);
        memcpy(vc, vp, sizeof(double) * 3 * n);
        double dt_prop = 0.0;
        for (int it = 0; it < 2; ++it) {
            if (it == 1 && !paper_rule)
                dt_prop = ora_pair_timestep(n, m, xc, vc, eta);
            ora_accjerk(n, m, xc, vc, ak, jk);
            ora_correct(n, h, xp, vp, a0, j0, ak, jk, xc, vc);
        }
        if (paper_rule)
            dt_prop = ora_paper_timestep(n, ak, jk, eta);
        memcpy(x, xc, sizeof(double) * 3 * n);
        memcpy(v, vc, sizeof(double) * 3 * n);
        memcpy(a0, ak, sizeof(double) * 3 * n);
        memcpy(j0, jk, sizeof(double) * 3 * n);
        *t = last ? t_end : *t + h;
        *dt_next = dt_prop;
        *steps += 1;
        status = ora_check_stop(n, m, x, v, stop_rules, r_eject);
    }
    return status;
}

/* ------------------------------------------------------------------------ */
/* Ensemble drivers: loop the single-system routines over a ragged ensemble  */
/* (body b of system s at flat index off[s] + b), optionally split over      */
/* nthreads host threads with a static partition by system.                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int s0, s1;
    const int *n_body;
    const long *off;
    const double *mass;
    double *pos, *vel, *acc, *jerk;
    double h;
    long nsteps;
    int n_corr, flags;
} fixed_job;

static void *fixed_worker(void *arg)
{
    fixed_job *jb = (fixed_job *)arg;
    for (int s = jb->s0; s < jb->s1; ++s) {
        long o = jb->off[s];
        ora_integrate_fixed(jb->n_body[s], jb->mass + o, jb->pos + 3 * o,
                            jb->vel + 3 * o, jb->acc + 3 * o, jb->jerk + 3 * o,
                            jb->h, jb->nsteps, jb->n_corr, jb->flags);
    }
    return NULL;
}

int ora_ensemble_fixed(int n_sys, const int *n_body, const double *mass,
                       double *pos, double *vel, double *acc, double *jerk,
                       double h, long nsteps, int n_corr, int flags,
                       int nthreads)
{
    if (n_sys < 0 || nthreads < 1)
        return -1;
    long *off = (long *)malloc(sizeof(long) * (size_t)(n_sys + 1));
    if (!off)
        return -2;
    off[0] = 0;
    for (int s = 0; s < n_sys; ++s) {
        if (n_body[s] < 1 || n_body[s] > ORA_MAX_BODIES) {
            free(off);
            return -1;
        }
        off[s + 1] = off[s] + n_body[s];
    }
    if (nthreads > n_sys)
        nthreads = n_sys > 0 ? n_sys : 1;
    pthread_t th[256];
    fixed_job jobs[256];
    if (nthreads > 256)
        nthreads = 256;
    for (int k = 0; k < nthreads; ++k) {
        jobs[k] = (fixed_job){(int)((long)n_sys * k / nthreads),
                              (int)((long)n_sys * (k + 1) / nthreads),
                              n_body, off, mass, pos, vel, acc, jerk, h,
                              nsteps, n_corr, flags};
    }
    for (int k = 1; k < nthreads; ++k)
        pthread_create(&th[k], NULL, fixed_worker, &jobs[k]);
    fixed_worker(&jobs[0]);
    for (int k = 1; k < nthreads; ++k)
        pthread_join(th[k], NULL);
    free(off);
    return 0;
}

int ora_ensemble_energy(int n_sys, const int *n_body, const double *mass,
                        const double *pos, const double *vel, double *energy,
                        double *angmom)
{
    long o = 0;
    for (int s = 0; s < n_sys; ++s) {
        int n = n_body[s];
        if (n < 1 || n > ORA_MAX_BODIES)
            return -1;
        ora_energy(n, mass + o, pos + 3 * o, vel + 3 * o, energy + s, angmom + 3 * s);
        o += n;
    }
    return 0;
}
