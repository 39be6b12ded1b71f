/* mvs_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow FP64 reference of the mixed-variable symplectic (MVS)
 * integrator of Section 2.2.3, for checking the HIP kernels.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product library never does, and the two share no code.
 *
 * The five sub-steps of Section 2.2.3 (Cartesian drift half step, kick half
 * step, Keplerian drift step, kick half step, Cartesian drift half step) are
 * the democratic heliocentric splitting of the N-body Hamiltonian (Duncan,
 * Levison & Lee 1998), with G = 1:
 *   variables: heliocentric planet positions Q_i = x_i - x_0 and barycentric
 *   velocities V_i = v_i - V (i >= 1), centre of mass X and its velocity V;
 *   H_kepler = sum_i m_i |V_i|^2 / 2 - m_0 m_i / |Q_i|  (each planet on a
 *              Kepler orbit about the star with mu = m_0),
 *   H_kick   = - sum_{1 <= i < j} m_i m_j / |Q_i - Q_j|  (planets only),
 *   H_drift  = |sum_i m_i V_i|^2 / (2 m_0)  (the star's reflex motion: its
 *              barycentric velocity is -sum_j m_j V_j / m_0, so every
 *              heliocentric Q_i moves by dt sum_j m_j V_j / m_0).
 * The kick evaluates the planet-planet accelerations at the current
 * positions every time.  The paper reuses the previous step's values
 * (Section 4.3.3); they are equal up to rounding, because the drifts move
 * all Q_i together.
 *
 * Kepler drift: for a bound orbit (1/a = 2/|r| - |v|^2/mu > 0) the change of
 * eccentric anomaly x over dt solves Kepler's equation in difference form
 *   n dt = x - (1 - |r|/a) sin x + (r.v / sqrt(mu a)) (1 - cos x),
 * n = sqrt(mu / a^3), by Newton iteration from x = n dt; then Lagrange's
 * f and g functions map (r, v) to the new state.  A planet whose
 * heliocentric orbit is not bound, or whose iteration does not converge in
 * 50 steps, stops the system (status ORA_UNBOUND).
 */
#include <math.h>
#include <stddef.h>

#define ORA_MVS_MAX 512
#define ORA_ACTIVE 0
#define ORA_DONE 1
#define ORA_NONFINITE 4
#define ORA_UNBOUND 7

/* Inertial (x, v) of n bodies (body 0 = star) -> Q, V of the planets
 * (rows 1..n-1 of Q and V; row 0 unused) and the centre of mass X, Vc. */
void ora_mvs_to_helio(int n, const double *m, const double *x, const double *v, double *Q,
                      double *V, double *X, double *Vc)
{
    double M = 0.0;
    for (int i = 0; i < n; ++i)
        M += m[i];
    for (int c = 0; c < 3; ++c) {
        double sx = 0.0, sv = 0.0;
        for (int i = 0; i < n; ++i) {
            sx += m[i] * x[3 * i + c];
            sv += m[i] * v[3 * i + c];
        }
        X[c] = sx / M;
        Vc[c] = sv / M;
    }
    for (int c = 0; c < 3; ++c) {
        Q[c] = 0.0;
        V[c] = 0.0;
    }
    for (int i = 1; i < n; ++i)
        for (int c = 0; c < 3; ++c) {
            Q[3 * i + c] = x[3 * i + c] - x[c];
            V[3 * i + c] = v[3 * i + c] - Vc[c];
        }
}

/* The inverse map: x_0 = X - sum m_i Q_i / M, x_i = x_0 + Q_i,
 * v_0 = Vc - sum m_i V_i / m_0, v_i = Vc + V_i. */
void ora_mvs_from_helio(int n, const double *m, const double *Q, const double *V,
                        const double *X, const double *Vc, double *x, double *v)
{
    double M = 0.0;
    for (int i = 0; i < n; ++i)
        M += m[i];
    for (int c = 0; c < 3; ++c) {
        double sq = 0.0, sp = 0.0;
        for (int i = 1; i < n; ++i) {
            sq += m[i] * Q[3 * i + c];
            sp += m[i] * V[3 * i + c];
        }
        x[c] = X[c] - sq / M;
        v[c] = Vc[c] - sp / m[0];
    }
    for (int i = 1; i < n; ++i)
        for (int c = 0; c < 3; ++c) {
            x[3 * i + c] = x[c] + Q[3 * i + c];
            v[3 * i + c] = Vc[c] + V[3 * i + c];
        }
}

/* Advance (r, v) along its Kepler orbit about mu by dt.  Returns 0, or -1
 * for an orbit that is not bound or an iteration that does not converge
 * (r, v untouched). */
int ora_kepler_drift(double mu, double *r, double *v, double dt)
{
    const double r0 = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const double rv = r[0] * v[0] + r[1] * v[1] + r[2] * v[2];
    const double alpha = 2.0 / r0 - v2 / mu;          /* 1 / a */
    if (!(alpha > 0.0))
        return -1;
    const double a = 1.0 / alpha;
    const double nmot = sqrt(mu / (a * a * a));
    const double ec = 1.0 - r0 / a;                   /* e cos E0 */
    const double es = rv / sqrt(mu * a);              /* e sin E0 */
    const double M = nmot * dt;
    double x = M;
    int ok = 0;
    for (int it = 0; it < 50; ++it) {
        const double s = sin(x), c = cos(x);
        const double F = x - ec * s + es * (1.0 - c) - M;
        const double dF = 1.0 - ec * c + es * s;
        const double dx = F / dF;
        x -= dx;
        if (fabs(dx) <= 1e-15 * (1.0 + fabs(x))) {
            ok = 1;
            break;
        }
    }
    if (!ok)
        return -1;
    const double s = sin(x), c = cos(x);
    const double f = 1.0 - (a / r0) * (1.0 - c);
    const double g = dt - (x - s) / nmot;
    const double rn = a * (1.0 - ec * c + es * s);
    const double fd = -sqrt(mu * a) * s / (rn * r0);
    const double gd = 1.0 - (a / rn) * (1.0 - c);
    for (int k = 0; k < 3; ++k) {
        const double rk = r[k], vk = v[k];
        r[k] = f * rk + g * vk;
        v[k] = fd * rk + gd * vk;
    }
    return 0;
}

/* Planet-planet accelerations at heliocentric positions Q (rows 1..n-1):
 * acc_i = sum_{j >= 1, j != i} m_j (Q_j - Q_i) / |Q_j - Q_i|^3, j ascending. */
void ora_mvs_kick_acc(int n, const double *m, const double *Q, double *acc)
{
    for (int c = 0; c < 3; ++c)
        acc[c] = 0.0;
    for (int i = 1; i < n; ++i) {
        double ai[3] = {0.0, 0.0, 0.0};
        for (int j = 1; j < n; ++j) {
            if (j == i)
                continue;
            double d[3];
            for (int c = 0; c < 3; ++c)
                d[c] = Q[3 * j + c] - Q[3 * i + c];
            const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            const double r3 = r2 * sqrt(r2);
            for (int c = 0; c < 3; ++c)
                ai[c] += m[j] * d[c] / r3;
        }
        for (int c = 0; c < 3; ++c)
            acc[3 * i + c] = ai[c];
    }
}

static void drift(int n, const double *m, double *Q, const double *V, double *X, const double *Vc,
                  double h)
{
    double P[3] = {0.0, 0.0, 0.0};
    for (int i = 1; i < n; ++i)
        for (int c = 0; c < 3; ++c)
            P[c] += m[i] * V[3 * i + c];
    for (int i = 1; i < n; ++i)
        for (int c = 0; c < 3; ++c)
            Q[3 * i + c] += h * P[c] / m[0];
    for (int c = 0; c < 3; ++c)
        X[c] += h * Vc[c];
}

static void kick(int n, const double *m, const double *Q, double *V, double h)
{
    double acc[3 * ORA_MVS_MAX];
    ora_mvs_kick_acc(n, m, Q, acc);
    for (int i = 1; i < n; ++i)
        for (int c = 0; c < 3; ++c)
            V[3 * i + c] += h * acc[3 * i + c];
}

/* One step of dt in the MVS variables.  Returns 0 or ORA_UNBOUND. */
int ora_mvs_step(int n, const double *m, double *Q, double *V, double *X, const double *Vc,
                 double dt)
{
    drift(n, m, Q, V, X, Vc, 0.5 * dt);
    kick(n, m, Q, V, 0.5 * dt);
    for (int i = 1; i < n; ++i)
        if (ora_kepler_drift(m[0], Q + 3 * i, V + 3 * i, dt) != 0)
            return ORA_UNBOUND;
    kick(n, m, Q, V, 0.5 * dt);
    drift(n, m, Q, V, X, Vc, 0.5 * dt);
    return 0;
}

/* nsteps fixed steps of dt on inertial (x, v), in place.  Returns
 * ORA_DONE, ORA_UNBOUND (state of the last completed step) or
 * ORA_NONFINITE; *steps_done gets the completed steps. */
int ora_integrate_mvs(int n, const double *m, double *x, double *v, double dt, long nsteps,
                      long *steps_done)
{
    if (n < 2 || n > ORA_MVS_MAX)
        return -1;
    double Q[3 * ORA_MVS_MAX], V[3 * ORA_MVS_MAX], X[3], Vc[3];
    ora_mvs_to_helio(n, m, x, v, Q, V, X, Vc);
    int status = ORA_DONE;
    long k = 0;
    for (; k < nsteps; ++k) {
        double Qs[3 * ORA_MVS_MAX], Vs[3 * ORA_MVS_MAX], Xs[3];
        for (int i = 0; i < 3 * n; ++i) {
            Qs[i] = Q[i];
            Vs[i] = V[i];
        }
        for (int c = 0; c < 3; ++c)
            Xs[c] = X[c];
        if (ora_mvs_step(n, m, Q, V, X, Vc, dt) != 0) {
            for (int i = 0; i < 3 * n; ++i) {
                Q[i] = Qs[i];
                V[i] = Vs[i];
            }
            for (int c = 0; c < 3; ++c)
                X[c] = Xs[c];
            status = ORA_UNBOUND;
            break;
        }
        int fin = 1;
        for (int i = 3; i < 3 * n; ++i)
            fin = fin && isfinite(Q[i]) && isfinite(V[i]);
        if (!fin) {
            status = ORA_NONFINITE;
            ++k;
            break;
        }
    }
    if (steps_done)
        *steps_done = k;
    ora_mvs_from_helio(n, m, Q, V, X, Vc, x, v);
    return status;
}
