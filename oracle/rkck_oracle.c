/* rkck_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 reference of the Runge-Kutta Cash-Karp integrator of
 * Sections 2.2.2 and 4.3.2, for checking the HIP kernels.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product library never does, and the two share no code.
 *
 * The method is the embedded 4(5) pair of Cash & Karp (ACM TOMS 16, 1990)
 * applied to y = (x, v), y' = (v, a(x)) with a(x) from Eq. 1 (G = 1):
 * six stages per step or trial step, each one acceleration evaluation.
 * Readings where the paper is silent:
 *  - the step advances with the fifth-order weights; the error estimate is
 *    the difference between the fifth- and fourth-order combinations;
 *  - adaptive control: with X and V the largest |x_i| and |v_i| of the
 *    system at the step's start, the error norm is
 *      E = max_i max(|dx_i| / (eps X), |dv_i| / (eps V))
 *    (|.| Euclidean per body).  E <= 1 accepts the step and proposes
 *    h * min(5, max(0.2, 0.9 E^(-1/5))) for the next one; E > 1 rejects it
 *    (state and time unchanged) and retries with h * max(0.1, 0.9 E^(-1/4)).
 *    The last step is shortened to land on t_end and leaves the proposed
 *    step unchanged; a step below 1e-12 |t_end| stalls the system.
 * Accelerations sum planet-planet pairs first and star pairs last (the
 * order of Section 4.2).
 */
#include <math.h>
#include <stddef.h>

#define ORA_RK_MAX 512
#define ORA_ACTIVE 0
#define ORA_DONE 1
#define ORA_NONFINITE 4
#define ORA_STALLED 5
#define ORA_MAXSTEPS 6

/* Cash & Karp (1990), Table 5: nodes, coupling coefficients, fifth-order
 * weights B and fourth-order weights BS. */
static const double A2[1] = {1.0 / 5.0};
static const double A3[2] = {3.0 / 40.0, 9.0 / 40.0};
static const double A4[3] = {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0};
static const double A5[4] = {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0};
static const double A6[5] = {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0,
                             44275.0 / 110592.0, 253.0 / 4096.0};
static const double B[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0, 512.0 / 1771.0};
static const double BS[6] = {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0, 13525.0 / 55296.0,
                             277.0 / 14336.0, 1.0 / 4.0};

/* Eq. 1: a_i = sum_j m_j (x_j - x_i) / |x_j - x_i|^3. */
void ora_rk_acc(int n, const double *m, const double *x, double *a)
{
    for (int k = 0; k < 3 * n; ++k)
        a[k] = 0.0;
    for (int pass = 0; pass < 2; ++pass)
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) {
                if ((pass == 0) != (i > 0))
                    continue;   /* pass 0: planet pairs; pass 1: star pairs */
                double d[3];
                for (int c = 0; c < 3; ++c)
                    d[c] = x[3 * j + c] - x[3 * i + c];
                const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                const double r3 = r2 * sqrt(r2);
                for (int c = 0; c < 3; ++c) {
                    a[3 * i + c] += m[j] * d[c] / r3;
                    a[3 * j + c] -= m[i] * d[c] / r3;
                }
            }
}

/* One Cash-Karp step of h from (x, v): fifth-order result (x5, v5) and the
 * error estimate (ex, ev); any output may alias nothing else. */
void ora_rkck_step(int n, const double *m, const double *x, const double *v, double h,
                   double *x5, double *v5, double *ex, double *ev)
{
    const double *coef[6] = {NULL, A2, A3, A4, A5, A6};
    double kx[6][3 * ORA_RK_MAX], kv[6][3 * ORA_RK_MAX];
    double xs[3 * ORA_RK_MAX], vs[3 * ORA_RK_MAX];
    const int m3 = 3 * n;
    for (int s = 0; s < 6; ++s) {
        for (int k = 0; k < m3; ++k) {
            double dx = 0.0, dv = 0.0;
            for (int j = 0; j < s; ++j) {
                dx += coef[s][j] * kx[j][k];
                dv += coef[s][j] * kv[j][k];
            }
            xs[k] = x[k] + h * dx;
            vs[k] = v[k] + h * dv;
        }
        for (int k = 0; k < m3; ++k)
            kx[s][k] = vs[k];
        ora_rk_acc(n, m, xs, kv[s]);
    }
    for (int k = 0; k < m3; ++k) {
        double sx = 0.0, sv = 0.0, ux = 0.0, uv = 0.0;
        for (int j = 0; j < 6; ++j) {
            sx += B[j] * kx[j][k];
            sv += B[j] * kv[j][k];
            ux += (B[j] - BS[j]) * kx[j][k];
            uv += (B[j] - BS[j]) * kv[j][k];
        }
        x5[k] = x[k] + h * sx;
        v5[k] = v[k] + h * sv;
        ex[k] = h * ux;
        ev[k] = h * uv;
    }
}

/* nsteps fixed steps of h, in place.  Returns ORA_DONE or ORA_NONFINITE. */
int ora_integrate_rkck_fixed(int n, const double *m, double *x, double *v, double h, long nsteps)
{
    if (n < 1 || n > ORA_RK_MAX)
        return -1;
    double x5[3 * ORA_RK_MAX], v5[3 * ORA_RK_MAX], ex[3 * ORA_RK_MAX], ev[3 * ORA_RK_MAX];
    for (long k = 0; k < nsteps; ++k) {
        ora_rkck_step(n, m, x, v, h, x5, v5, ex, ev);
        for (int i = 0; i < 3 * n; ++i) {
            x[i] = x5[i];
            v[i] = v5[i];
        }
    }
    for (int i = 0; i < 3 * n; ++i)
        if (!isfinite(x[i]) || !isfinite(v[i]))
            return ORA_NONFINITE;
    return ORA_DONE;
}

static double norm3(const double *p) { return sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]); }

/* The error norm E of a trial step (see the header). */
double ora_rkck_error_norm(int n, const double *x, const double *v, const double *ex,
                           const double *ev, double eps)
{
    double X = 0.0, V = 0.0, E = 0.0;
    for (int i = 0; i < n; ++i) {
        X = fmax(X, norm3(x + 3 * i));
        V = fmax(V, norm3(v + 3 * i));
    }
    for (int i = 0; i < n; ++i) {
        E = fmax(E, norm3(ex + 3 * i) / (eps * X));
        E = fmax(E, norm3(ev + 3 * i) / (eps * V));
    }
    return E;
}

/* Adaptive integration from *t to t_end, in place; *dt is the first trial
 * step on entry and the proposed next step on return.  Returns the status;
 * *steps counts accepted steps, *rejects rejected trials. */
int ora_integrate_rkck_adaptive(int n, const double *m, double *x, double *v, double *t,
                                double t_end, double eps, double *dt, long max_steps,
                                long *steps, long *rejects)
{
    if (n < 1 || n > ORA_RK_MAX || !(*dt > 0.0) || !(eps > 0.0))
        return -1;
    double x5[3 * ORA_RK_MAX], v5[3 * ORA_RK_MAX], ex[3 * ORA_RK_MAX], ev[3 * ORA_RK_MAX];
    long acc = 0, rej = 0;
    int status = ORA_ACTIVE;
    double h_next = *dt;
    while (status == ORA_ACTIVE) {
        if (*t >= t_end) {
            *t = t_end;
            status = ORA_DONE;
            break;
        }
        if (acc >= max_steps) {
            status = ORA_MAXSTEPS;
            break;
        }
        if (!(h_next >= 1e-12 * fabs(t_end))) {
            status = ORA_STALLED;
            break;
        }
        int last = 0;
        double h = h_next;
        if (*t + h >= t_end) {
            h = t_end - *t;
            last = 1;
        }
        ora_rkck_step(n, m, x, v, h, x5, v5, ex, ev);
        const double E = ora_rkck_error_norm(n, x, v, ex, ev, eps);
        if (!(E <= 1.0)) {
            if (!isfinite(E)) {
                status = ORA_NONFINITE;
                break;
            }
            h_next = h * fmax(0.1, 0.9 * pow(E, -0.25));
            ++rej;
            continue;
        }
        for (int i = 0; i < 3 * n; ++i) {
            x[i] = x5[i];
            v[i] = v5[i];
        }
        *t = last ? t_end : *t + h;
        ++acc;
        /* a step shortened onto t_end leaves the proposal as it was */
        if (!last)
            h_next = h * (E > 0.0 ? fmin(5.0, fmax(0.2, 0.9 * pow(E, -0.2))) : 5.0);
    }
    *dt = h_next;
    *steps = acc;
    *rejects = rej;
    return status;
}
