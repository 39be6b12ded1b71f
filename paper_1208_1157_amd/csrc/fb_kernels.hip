// fb_kernels.hip -- gfx950 kernels of libfewbody.
//
// FP64 fourth-order time-symmetrised Hermite P(EC)^2 steps of many
// independent few-body systems (Swarm-NG, arXiv:1208.1157: Eq. 1 and its
// time derivative for the pair forces, Eq. 3 predictor, Eq. 4 corrector
// applied twice per step as in Algorithm 2, many steps per launch as in
// Algorithm 1).  All arithmetic is FP64 on the vector ALUs; the pair sums are
// not a dense contraction, so no MFMA is used.
//
// Two lane mappings (both read the bucket's structure-of-arrays state with
// consecutive lanes on consecutive slots):
//   SPL  one system per lane.  The whole system lives in VGPRs for the whole
//        step loop; every pair is evaluated once (Newton's third law), no
//        cross-lane traffic.  Used for small n.
//   BPL  one body per lane, floor(64/n) systems per wavefront (lane = body *
//        S + system).  Each lane evaluates its body's n-1 interactions with
//        partner positions/velocities read from the wave's LDS slice; no
//        reduction is needed and every lane does useful work.
// In both, each body sums its planet partners in ascending order and the
// star last (Section 4.2).
//
// The corrector is Eq. 4 read with coefficient 3/20, a (dt)^3 jerk term and
// the predicted state (xp, vp) as the base of every correction:
//   x1 = xp - 3/20 (a0 - ak) h^2 - (7 j0 + 2 jk) h^3 / 60
//   v1 = vp - 1/2 (a0 - ak) h - (5 j0 + jk) h^2 / 12
// The a0/j0 parts are folded into per-step bases, so each correction costs
// four FMAs per component and does not need the corrected velocity.
#include "fb_internal.h"

#include <algorithm>
#include <climits>

// Partner-loop unroll of the body-per-lane evaluation: full unrolling lets
// the scheduler hoist every partner's LDS loads and costs occupancy.
#ifndef FB_BPL_UNROLL
#define FB_BPL_UNROLL 1
#endif
// Pairs per scheduling group in the system-per-lane evaluation of n >= 5.
#ifndef FB_SPL_PAIR_GROUP
#define FB_SPL_PAIR_GROUP 2
#endif
// Waves per SIMD the register allocator targets for the body-per-lane and
// persistent kernels: 3 (168 VGPRs) leaves the adaptive variants unspilled and
// measured faster than 4 (128 VGPRs, with spills) in fixed and adaptive runs.
#ifndef FB_BPL_WAVES
#define FB_BPL_WAVES 3
#endif

namespace fb {
namespace {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

// LDS exchange among the lanes of one wavefront: order this wave's LDS
// writes before its subsequent reads (no workgroup barrier needed: every
// exchange stays inside one wavefront's slice).
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1/sqrt(x): hardware estimate y (v_rsq_f64, relative error ~6e-8 on
// gfx950) refined by one third-order step of the series
// 1/sqrt(x) = y (1 - e)^(-1/2) = y (1 + e/2 + 3e^2/8 + ...), e = 1 - x y^2,
// whose truncation (~e^3) is far below FP64 rounding.
__device__ __forceinline__ double rsqrt_nr(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    const double p = fma(0.375, e, 0.5);
    return fma(y * e, p, y);
}

__device__ __forceinline__ bool finite3(const double (&p)[3])
{
    return __builtin_isfinite(p[0]) && __builtin_isfinite(p[1]) && __builtin_isfinite(p[2]);
}

// Wave-uniform copies (scalar registers) of values every lane holds alike:
// tests on them are scalar branches rather than exec-mask changes.
__device__ __forceinline__ int uniform_i(const int v)
{
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ long long uniform_ll(const long long v)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(v & 0xffffffffll));
    const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}

__device__ __forceinline__ double uniform_d(const double v)
{
    return __longlong_as_double(uniform_ll(__double_as_longlong(v)));
}

__device__ __forceinline__ StepParams uniform_params(const StepParams &P)
{
    StepParams u;
    u.adaptive = uniform_i(P.adaptive);
    u.stop_rules = uniform_i(P.stop_rules);
    u.eta = uniform_d(P.eta);
    u.r_eject = uniform_d(P.r_eject);
    u.max_steps = uniform_ll(P.max_steps);
    u.quantum = uniform_i(P.quantum);
    u.pad = 0;
    return u;
}

// Step coefficients of the predictor (Eq. 3) and corrector (Eq. 4).
struct Coef {
    double h, hh2, hhh6;       // predictor: h, h^2/2, h^3/6
    double bxa, bxj, bva, bvj; // bases: -3/20 h^2, -7/60 h^3, -h/2, -5/12 h^2
    double cxa, cxj, cva, cvj; // corrections: 3/20 h^2, -h^3/30, h/2, -h^2/12
};

__device__ __forceinline__ Coef make_coef(double h)
{
    Coef k;
    const double h2 = h * h, h3 = h2 * h;
    k.h = h;
    k.hh2 = 0.5 * h2;
    k.hhh6 = h3 * (1.0 / 6.0);
    k.cxa = 0.15 * h2;
    k.cxj = h3 * (-1.0 / 30.0);
    k.cva = 0.5 * h;
    k.cvj = h2 * (-1.0 / 12.0);
    k.bxa = -k.cxa;
    k.bxj = h3 * (-7.0 / 60.0);
    k.bva = -k.cva;
    k.bvj = h2 * (-5.0 / 12.0);
    return k;
}

// Predicted state and the per-step bases of the corrector for one component.
__device__ __forceinline__ void predict_comp(const Coef &k, double x, double v, double a,
                                             double j, double &xp, double &vp, double &bx,
                                             double &bv)
{
    xp = fma(k.hhh6, j, fma(k.hh2, a, fma(k.h, v, x)));
    vp = fma(k.hh2, j, fma(k.h, a, v));
    bx = fma(k.bxj, j, fma(k.bxa, a, xp));
    bv = fma(k.bvj, j, fma(k.bva, a, vp));
}

// One correction of one component from the latest evaluation (ak, jk).
__device__ __forceinline__ void correct_comp(const Coef &k, double bx, double bv, double ak,
                                             double jk, double &xc, double &vc)
{
    xc = fma(k.cxj, jk, fma(k.cxa, ak, bx));
    vc = fma(k.cvj, jk, fma(k.cva, ak, bv));
}

// One wavefront's LDS slice: the current evaluation state of its 64 lanes
// (as 16-byte pairs so a partner costs three ds_read_b128 and one b64), and
// per lane its mass beside a reduction scratch value, so every row of a
// partner sits at the same 16-byte slot offset.
struct BplLds {
    double2 xy[64];
    double2 zvx[64];
    double2 vyvz[64];
    double2 mr[64];   // (mass, reduction scratch)
};

// System-per-lane steps of at least this many bodies park the corrector
// bases (6 doubles per body, idle during each evaluation) in the wavefront's
// LDS slice, so the evaluation's working set (12 doubles per body) stays in
// VGPRs.
#ifndef FB_SPL_LDS_MIN
#define FB_SPL_LDS_MIN 6
#endif

// Rows parked after the bases by the adaptive step loop (n <= kMaxSplAdv):
// the step size and the system's clock (t, t_end, carried step, run steps,
// steps, status, last step).
constexpr int kSplParkClock = 8;

// LDS bytes per wavefront a system-per-lane step of n bodies uses.
__host__ __device__ constexpr size_t spl_lds_bytes(int n)
{
    return n >= FB_SPL_LDS_MIN
               ? (size_t)(6 * n + (n <= kMaxSplAdv ? kSplParkClock : 0)) * 64 * sizeof(double)
               : 0;
}

// Per-wavefront LDS stride of the system-per-lane fused class, whose waves
// may run either kind of tile side by side in one workgroup: large enough
// for the body-per-lane slice and for the largest parked bases.
constexpr size_t kWideLdsStride = 6 * kMaxSplBodies * 64 * sizeof(double);
static_assert(kWideLdsStride >= sizeof(BplLds), "wide LDS stride too small");
static_assert(kWideLdsStride >= spl_lds_bytes(kMaxSplAdv) &&
                  kWideLdsStride >= spl_lds_bytes(kMaxSplBodies), "wide LDS stride too small");

// This wavefront's slice of its workgroup's dynamic LDS, reached through
// the module-level symbol (not a pointer argument) so separately compiled
// tile functions still address LDS directly.  PACKED is the slice size when
// every wave of the launch runs the same kind of tile; WIDE selects the
// common stride of the system-per-lane fused class.
template <size_t PACKED, bool WIDE>
__device__ __forceinline__ char *wave_lds_base()
{
    extern __shared__ char fb_dyn_lds[];
    return fb_dyn_lds + (size_t)(threadIdx.x >> 6) * (WIDE ? kWideLdsStride : PACKED);
}

// ---------------------------------------------------------------------------
// per-system clock (Algorithm 1's loop control)
// ---------------------------------------------------------------------------
struct Clock {
    double t, t_end, dt, dtn, t0;
    long long k, nfull, steps;
    int status;
};

__device__ __forceinline__ Clock load_clock(const Bucket &B, int s)
{
    Clock c;
    c.t = B.t[s];
    c.t_end = B.t_end[s];
    c.dt = B.dt[s];
    c.dtn = B.dtn[s];
    c.t0 = B.t0run[s];
    c.k = B.krun[s];
    c.nfull = B.nfull[s];
    c.steps = B.steps[s];
    c.status = B.status[s];
    return c;
}

__device__ __forceinline__ void store_clock(const Bucket &B, int s, const Clock &c)
{
    B.t[s] = c.t;
    B.dtn[s] = c.dtn;
    B.krun[s] = c.k;
    B.steps[s] = c.steps;
    B.status[s] = c.status;
}

// Size of the next step, or false (with the status updated) if the system
// takes no further step.
__device__ __forceinline__ bool plan_step(Clock &c, const StepParams &P, double &h, bool &last)
{
    if (c.status != ST_ACTIVE)
        return false;
    if (P.adaptive) {
        if (!(c.t < c.t_end)) {
            c.status = ST_DONE;
            return false;
        }
        if (c.steps >= P.max_steps) {
            c.status = ST_MAXSTEPS;
            return false;
        }
        if (__builtin_isnan(c.dtn)) {
            c.status = ST_NONFINITE;
            return false;
        }
        if (!(c.dtn >= 1e-12 * fabs(c.t_end))) {
            c.status = ST_STALLED;
            return false;
        }
        last = c.t + c.dtn >= c.t_end;
        h = last ? c.t_end - c.t : c.dtn;
        return true;
    }
    if (c.steps >= P.max_steps) {
        c.status = ST_MAXSTEPS;
        return false;
    }
    if (c.k < c.nfull) {
        h = c.dt;
        last = false;
        return true;
    }
    const double rem = c.t_end - c.t;
    if (rem * c.dt > 1e-9 * c.dt * c.dt) {   // remainder in the direction of dt
        h = rem;
        last = true;
        return true;
    }
    c.t = c.t_end;
    c.status = ST_DONE;
    return false;
}

__device__ __forceinline__ void finish_step(Clock &c, const StepParams &P, bool last, double h,
                                            double dt_prop)
{
    c.steps += 1;
    if (P.adaptive) {
        c.t = last ? c.t_end : c.t + h;
        c.dtn = dt_prop;
        if (last)
            c.status = ST_DONE;
        return;
    }
    if (last) {
        c.t = c.t_end;
        c.status = ST_DONE;
        return;
    }
    c.k += 1;
    c.t = fma((double)c.k, c.dt, c.t0);
    if (c.k >= c.nfull) {
        const double rem = c.t_end - c.t;
        if (!(rem * c.dt > 1e-9 * c.dt * c.dt)) {
            c.t = c.t_end;
            c.status = ST_DONE;
        }
    }
}

__device__ __forceinline__ int status_of_flags(int fl)
{
    return (fl & 1) ? ST_NONFINITE : (fl & 2) ? ST_ENCOUNTER : (fl & 4) ? ST_EJECTED : ST_ACTIVE;
}

// Adaptive-step forms of plan_step and finish_step (the same tests in the
// same order) as selects rather than branches, for a wave that runs alone on
// its SIMD, where every branch and exec-mask change is latency on the step's
// critical path.  A lane whose system is not active keeps its clock.
__device__ __forceinline__ bool plan_step_adaptive(Clock &c, const StepParams &P, double &h,
                                                   bool &last)
{
    const bool running = c.status == ST_ACTIVE;
    // every test evaluated, then the first that holds wins
    const bool done = !(c.t < c.t_end);
    const bool maxed = c.steps >= P.max_steps;
    const bool nonfinite = __builtin_isnan(c.dtn);
    const bool stalled = !(c.dtn >= 1e-12 * fabs(c.t_end));
    int ns = stalled ? ST_STALLED : ST_ACTIVE;
    ns = nonfinite ? ST_NONFINITE : ns;
    ns = maxed ? ST_MAXSTEPS : ns;
    ns = done ? ST_DONE : ns;
    c.status = running ? ns : c.status;
    last = c.t + c.dtn >= c.t_end;
    h = last ? c.t_end - c.t : c.dtn;
    return running && ns == ST_ACTIVE;
}

__device__ __forceinline__ void finish_step_adaptive(Clock &c, const bool act, const bool last,
                                                     const double h, const double dt_prop,
                                                     const int fl)
{
    c.steps += act ? 1 : 0;
    c.t = act ? (last ? c.t_end : c.t + h) : c.t;
    c.dtn = act ? dt_prop : c.dtn;
    const int st = fl ? status_of_flags(fl) : (last ? ST_DONE : c.status);
    c.status = act ? st : c.status;
}

// ---------------------------------------------------------------------------
// system-per-lane (SPL)
// ---------------------------------------------------------------------------

// Pair (i, j): r = x_j - x_i, u = v_j - v_i, A = r/|r|^3,
// J = u/|r|^3 - 3 (r.u)/|r|^2 A; body i gains m_j (A, J), body j loses
// m_i (A, J).  With TS, also track max over pairs of
// (|u|^2 + 3 (r.u)^2/|r|^2) / |r|^2 = (|j_ij| / |a_ij|)^2 of the pair's
// two-body relative motion (the step rule's quantity).
template <int N, bool TS>
__device__ __forceinline__ void spl_pair(const int i, const int j, const double (&m)[N],
                                         const double (&x)[N][3], const double (&v)[N][3],
                                         double (&a)[N][3], double (&jk)[N][3], double &wmax)
{
    const double rx = x[j][0] - x[i][0], ry = x[j][1] - x[i][1], rz = x[j][2] - x[i][2];
    const double ux = v[j][0] - v[i][0], uy = v[j][1] - v[i][1], uz = v[j][2] - v[i][2];
    const double r2 = fma(rz, rz, fma(ry, ry, rx * rx));
    const double ru = fma(rz, uz, fma(ry, uy, rx * ux));
    const double ri = rsqrt_nr(r2);
    const double ri2 = ri * ri;
    const double ri3 = ri2 * ri;
    const double al = 3.0 * ru * ri2;
    // J / |r|^-3 = u - 3 (r.u)/|r|^2 r; masses folded into |r|^-3
    const double wx = fma(-al, rx, ux), wy = fma(-al, ry, uy), wz = fma(-al, rz, uz);
    const double mj3 = m[j] * ri3, mi3 = m[i] * ri3;
    a[i][0] = fma(mj3, rx, a[i][0]);
    a[i][1] = fma(mj3, ry, a[i][1]);
    a[i][2] = fma(mj3, rz, a[i][2]);
    a[j][0] = fma(-mi3, rx, a[j][0]);
    a[j][1] = fma(-mi3, ry, a[j][1]);
    a[j][2] = fma(-mi3, rz, a[j][2]);
    jk[i][0] = fma(mj3, wx, jk[i][0]);
    jk[i][1] = fma(mj3, wy, jk[i][1]);
    jk[i][2] = fma(mj3, wz, jk[i][2]);
    jk[j][0] = fma(-mi3, wx, jk[j][0]);
    jk[j][1] = fma(-mi3, wy, jk[j][1]);
    jk[j][2] = fma(-mi3, wz, jk[j][2]);
    if (TS) {
        const double u2 = fma(uz, uz, fma(uy, uy, ux * ux));
        wmax = fmax(wmax, fma(al, ru, u2) * ri2);
        // Keep the running maximum a serial chain through the pairs: left
        // free, the compiler rebalances it into a tree at the end, which
        // keeps every pair's inputs live and spills systems of n >= 6.
        __asm__ __volatile__("" : "+v"(wmax));
    }
}

// Acceleration and jerk of every body: planet-planet pairs first, then the
// star's pairs, so each planet adds the star's contribution last.
template <int N, bool TS>
__device__ __forceinline__ void spl_accjerk(const double (&m)[N], const double (&x)[N][3],
                                            const double (&v)[N][3], double (&a)[N][3],
                                            double (&jk)[N][3], double &wmax)
{
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a[b][c] = 0.0;
            jk[b][c] = 0.0;
        }
    // For larger systems, scheduling barriers between groups of pairs keep
    // the scheduler from interleaving (and keeping live) every pair's
    // temporaries at once, which would spill the system's state.
    constexpr int kGroup = N <= 4 ? 1 << 20 : FB_SPL_PAIR_GROUP;
#pragma unroll
    for (int i = 1; i < N; ++i)
#pragma unroll
        for (int j = i + 1; j < N; ++j) {
            spl_pair<N, TS>(i, j, m, x, v, a, jk, wmax);
            if (((i - 1) * (2 * N - i - 2) / 2 + (j - i)) % kGroup == 0)
                __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
    for (int j = 1; j < N; ++j) {
        spl_pair<N, TS>(0, j, m, x, v, a, jk, wmax);
        if (j % kGroup == 0)
            __builtin_amdgcn_sched_barrier(0);
    }
}

// This lane's parking area: [6N + kSplParkClock][64] doubles, lane fastest.
template <int N, bool WIDE>
__device__ __forceinline__ double *spl_park()
{
    return reinterpret_cast<double *>(wave_lds_base<spl_lds_bytes(N), WIDE>()) + (threadIdx.x & 63);
}

// One P(EC)^2 step of size h.  On entry (a, jk) hold the carried a0, j0; on
// exit (x, v) are the corrected state and (a, jk) the last evaluation.
// Returns the step-rule quantity of the last evaluation (TS only).  With
// RELOAD (parked steps only) the caller has parked h in row 6N and the step
// coefficients are rebuilt from it after each evaluation instead of being
// kept in registers through it.
template <int N, bool TS, bool WIDE, bool RELOAD = false>
__device__ __forceinline__ double spl_step(const double (&m)[N], double (&x)[N][3],
                                           double (&v)[N][3], double (&a)[N][3],
                                           double (&jk)[N][3], const Coef &k0)
{
    constexpr bool kPark = N >= FB_SPL_LDS_MIN;
    static_assert(!RELOAD || kPark, "coefficient reload needs the parking area");
    double *park = spl_park<N, WIDE>();
    Coef k = k0;
    double bx[N][3], bv[N][3], xc[N][3], vc[N][3];
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            predict_comp(k, x[b][c], v[b][c], a[b][c], jk[b][c], xc[b][c], vc[b][c], bx[b][c],
                         bv[b][c]);
            if (kPark) {
                park[(6 * b + c) * 64] = bx[b][c];
                park[(6 * b + 3 + c) * 64] = bv[b][c];
            }
        }
    // The clobbers keep the compiler from forwarding the parked values
    // (which would keep them in registers) or hoisting their reloads above
    // the evaluation.
    if (kPark)
        __asm__ __volatile__("" ::: "memory");
    double w = 0.0;
    spl_accjerk<N, false>(m, xc, vc, a, jk, w);
    if (kPark)
        __asm__ __volatile__("" ::: "memory");
    if (RELOAD)
        k = make_coef(park[6 * N * 64]);
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (kPark) {
                bx[b][c] = park[(6 * b + c) * 64];
                bv[b][c] = park[(6 * b + 3 + c) * 64];
            }
            correct_comp(k, bx[b][c], bv[b][c], a[b][c], jk[b][c], xc[b][c], vc[b][c]);
        }
    if (kPark)
        __asm__ __volatile__("" ::: "memory");
    spl_accjerk<N, TS>(m, xc, vc, a, jk, w);
    if (kPark)
        __asm__ __volatile__("" ::: "memory");
    if (RELOAD)
        k = make_coef(park[6 * N * 64]);
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (kPark) {
                bx[b][c] = park[(6 * b + c) * 64];
                bv[b][c] = park[(6 * b + 3 + c) * 64];
            }
            correct_comp(k, bx[b][c], bv[b][c], a[b][c], jk[b][c], xc[b][c], vc[b][c]);
            x[b][c] = xc[b][c];
            v[b][c] = vc[b][c];
        }
    return w;
}

// Stop-rule flags after a committed step: bit 0 non-finite, bit 1 two
// planets within one mutual Hill radius, bit 2 a planet beyond r_eject.
// The Hill test sep < ((m_i+m_j)/(3 m0))^(1/3) (r_i+r_j)/2 (r the astrocentric
// distance) is evaluated without roots as
// sep^6 < ((m_i+m_j)/(24 m0))^2 ((r_i+r_j)^2)^3.
__device__ __forceinline__ bool hill_close(double sep2, double mi, double mj, double inv24m0,
                                           double ri, double rj)
{
    const double mu = (mi + mj) * inv24m0;
    const double w = (ri + rj) * (ri + rj);
    return sep2 * sep2 * sep2 < mu * mu * (w * w * w);
}

template <int N>
__device__ __forceinline__ int spl_stop_flags(const double (&m)[N], const double (&x)[N][3],
                                              const double (&v)[N][3], const StepParams &P)
{
    bool fin = true;
#pragma unroll
    for (int b = 0; b < N; ++b)
        fin = fin && finite3(x[b]) && finite3(v[b]);
    if (!fin)
        return 1;
    double r[N];
    r[0] = 0.0;
#pragma unroll
    for (int i = 1; i < N; ++i) {
        const double dx = x[i][0] - x[0][0], dy = x[i][1] - x[0][1], dz = x[i][2] - x[0][2];
        r[i] = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
    }
    int fl = 0;
    if (P.stop_rules & 1) {
        const double inv24m0 = 1.0 / (24.0 * m[0]);
#pragma unroll
        for (int i = 1; i < N; ++i)
#pragma unroll
            for (int j = i + 1; j < N; ++j) {
                const double dx = x[i][0] - x[j][0], dy = x[i][1] - x[j][1],
                             dz = x[i][2] - x[j][2];
                const double sep2 = fma(dz, dz, fma(dy, dy, dx * dx));
                if (hill_close(sep2, m[i], m[j], inv24m0, r[i], r[j]))
                    fl |= 2;
            }
    }
    if (P.stop_rules & 2) {
#pragma unroll
        for (int i = 1; i < N; ++i)
            if (r[i] > P.r_eject)
                fl |= 4;
    }
    return fl;
}

// Eq. 5 (Section 4.3.1): tau [sum_i |j_i|^2 / |a_i|^2]^(-1/2) from the
// accelerations and jerks that start the next step, summed in body order.
template <int N>
__device__ __forceinline__ double paper_dt(const double (&a)[N][3], const double (&jk)[N][3],
                                           double tau)
{
    double sum = 0.0;
#pragma unroll
    for (int b = 0; b < N; ++b) {
        const double aa = fma(a[b][2], a[b][2], fma(a[b][1], a[b][1], a[b][0] * a[b][0]));
        const double jj = fma(jk[b][2], jk[b][2], fma(jk[b][1], jk[b][1], jk[b][0] * jk[b][0]));
        sum += jj / aa;
    }
    return tau * rsqrt_nr(sum);
}

// Integrate one system (one lane) for at most P.quantum steps.
template <int N, bool ADV, bool WIDE>
__device__ __forceinline__ void spl_run(const Bucket &B, const int slot, const StepParams &P)
{
    Clock c = load_clock(B, slot);
    if (c.status != ST_ACTIVE)
        return;
    const size_t pitch = B.pitch;
    const double *st = B.st;
    double m[N], x[N][3], v[N][3], a[N][3], jk[N][3];
#pragma unroll
    for (int b = 0; b < N; ++b) {
        m[b] = st[(R_M * N + b) * pitch + slot];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            x[b][cc] = st[((R_X + cc) * N + b) * pitch + slot];
            v[b][cc] = st[((R_V + cc) * N + b) * pitch + slot];
            a[b][cc] = st[((R_A + cc) * N + b) * pitch + slot];
            jk[b][cc] = st[((R_J + cc) * N + b) * pitch + slot];
        }
    }
    if (!ADV) {
        // Fixed step.  Segment 0 runs the run's whole steps with no per-step
        // bookkeeping; segment 1 the shortened final step, if one is due.
        // One loop serves both so the step body is instantiated once.
        int budget = P.quantum;
#pragma unroll 1
        for (int seg = 0; seg < 2 && c.status == ST_ACTIVE && budget > 0; ++seg) {
            long long cnt = 0;
            double h = c.dt;
            if (seg == 0) {
                cnt = c.nfull - c.k;
                cnt = cnt < 0 ? 0 : cnt;
            } else {
                const double rem = c.t_end - c.t;
                if (rem * c.dt > 1e-9 * c.dt * c.dt) {
                    cnt = 1;
                    h = rem;
                } else {
                    c.t = c.t_end;
                    c.status = ST_DONE;
                }
            }
            cnt = min(cnt, (long long)budget);
            cnt = min(cnt, P.max_steps - c.steps);
            const int nrun = cnt > 0 ? (int)cnt : 0;
            const Coef k = make_coef(h);
            constexpr int kStepUnroll = N <= 4 ? 2 : 1;
#pragma unroll kStepUnroll
            for (int q = 0; q < nrun; ++q)
                (void)spl_step<N, false, WIDE>(m, x, v, a, jk, k);
            budget -= nrun;
            c.steps += nrun;
            if (seg == 0) {
                c.k += nrun;
                if (nrun > 0)
                    c.t = fma((double)c.k, c.dt, c.t0);
                if (c.k >= c.nfull) {
                    const double rem = c.t_end - c.t;
                    if (!(rem * c.dt > 1e-9 * c.dt * c.dt)) {
                        c.t = c.t_end;
                        c.status = ST_DONE;
                    }
                }
            } else if (nrun > 0) {
                c.t = c.t_end;
                c.status = ST_DONE;
            }
            if (c.status == ST_ACTIVE && c.steps >= P.max_steps)
                c.status = ST_MAXSTEPS;
        }
    } else {
        // Parked steps also park the step size and the clock across the step
        // (rows 6N..6N+7), so the evaluations keep only the system in VGPRs.
        constexpr bool kParkClock = N >= FB_SPL_LDS_MIN;
        double *pc = kParkClock ? spl_park<N, WIDE>() + 6 * N * 64 : nullptr;
        for (int q = 0; q < P.quantum; ++q) {
            double h = 0.0;
            bool last = false;
            if (!plan_step(c, P, h, last))
                break;
            if constexpr (kParkClock) {
                pc[0] = h;
                pc[64] = c.t;
                pc[2 * 64] = c.t_end;
                pc[3 * 64] = c.dtn;
                pc[4 * 64] = __longlong_as_double(c.k);
                pc[5 * 64] = __longlong_as_double(c.steps);
                pc[6 * 64] = (double)c.status;
                pc[7 * 64] = last ? 1.0 : 0.0;
                __asm__ __volatile__("" ::: "memory");
            }
            const double w = spl_step<N, true, WIDE, kParkClock>(m, x, v, a, jk, make_coef(h));
            if constexpr (kParkClock) {
                __asm__ __volatile__("" ::: "memory");
                h = pc[0];
                c.t = pc[64];
                c.t_end = pc[2 * 64];
                c.dtn = pc[3 * 64];
                c.k = __double_as_longlong(pc[4 * 64]);
                c.steps = __double_as_longlong(pc[5 * 64]);
                c.status = (int)pc[6 * 64];
                last = pc[7 * 64] != 0.0;
            }
            double dtp = P.adaptive == 2 ? paper_dt<N>(a, jk, P.eta) : P.eta * rsqrt_nr(w);
            finish_step(c, P, last, h, dtp);
            const int fl = spl_stop_flags<N>(m, x, v, P);
            if (fl)
                c.status = status_of_flags(fl);
            if (c.status != ST_ACTIVE)
                break;
        }
    }
    if (!ADV) {
        bool fin = true;
#pragma unroll
        for (int b = 0; b < N; ++b)
            fin = fin && finite3(x[b]) && finite3(v[b]);
        if (!fin)
            c.status = ST_NONFINITE;
    }
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            B.st[((R_X + cc) * N + b) * pitch + slot] = x[b][cc];
            B.st[((R_V + cc) * N + b) * pitch + slot] = v[b][cc];
            B.st[((R_A + cc) * N + b) * pitch + slot] = a[b][cc];
            B.st[((R_J + cc) * N + b) * pitch + slot] = jk[b][cc];
        }
    store_clock(B, slot, c);
}

// ---------------------------------------------------------------------------
// body-per-lane (BPL)
// ---------------------------------------------------------------------------


// LDS slot of the k-th planet partner (0 <= k < N-2, the other planets in
// ascending order) of body b of system s, with own = b S (the star lane
// passes 64, past every body): (k + 1) S + s, moved one body up from b on.
// The body offset (k + 1) S is uniform, so the slot costs a compare, a select
// and an add per partner.
template <int N>
__device__ __forceinline__ int partner_slot(const int k, const int s, const int own)
{
    constexpr int S = 64 / N;
    const int ks = (k + 1) * S;
    return s + ks + (ks >= own ? S : 0);
}

// A partner's evaluation state as read from the wavefront's LDS slice.
struct Partner {
    double2 p0, p1, p2;   // (x, y), (z, vx), (vy, vz)
    double mj;
};

__device__ __forceinline__ Partner bpl_partner(const BplLds &L, const int idx)
{
    return Partner{L.xy[idx], L.zvx[idx], L.vyvz[idx], L.mr[idx].x};
}

// One interaction of body i (this lane) with partner P: adds m_j A and m_j J
// (Eq. 1 and its time derivative).
template <bool TS>
__device__ __forceinline__ void bpl_interact_p(const Partner &Pj, const double (&xi)[3],
                                               const double (&vi)[3], double (&a)[3],
                                               double (&jk)[3], double &wmax)
{
    const double2 p0 = Pj.p0, p1 = Pj.p1, p2 = Pj.p2;
    const double mj = Pj.mj;
    const double rx = p0.x - xi[0], ry = p0.y - xi[1], rz = p1.x - xi[2];
    const double ux = p1.y - vi[0], uy = p2.x - vi[1], uz = p2.y - vi[2];
    const double r2 = fma(rz, rz, fma(ry, ry, rx * rx));
    const double ru = fma(rz, uz, fma(ry, uy, rx * ux));
    const double ri = rsqrt_nr(r2);
    const double ri2 = ri * ri;
    const double mr3 = mj * (ri2 * ri);
    const double al = 3.0 * ru * ri2;
    a[0] = fma(mr3, rx, a[0]);
    a[1] = fma(mr3, ry, a[1]);
    a[2] = fma(mr3, rz, a[2]);
    jk[0] = fma(mr3, fma(-al, rx, ux), jk[0]);
    jk[1] = fma(mr3, fma(-al, ry, uy), jk[1]);
    jk[2] = fma(mr3, fma(-al, rz, uz), jk[2]);
    if (TS) {
        const double u2 = fma(uz, uz, fma(uy, uy, ux * ux));
        wmax = fmax(wmax, fma(al, ru, u2) * ri2);
    }
}

// One interaction of body i (this lane) with the partner stored at LDS index
// idx.
template <bool TS>
__device__ __forceinline__ void bpl_interact(const BplLds &L, const int idx,
                                             const double (&xi)[3], const double (&vi)[3],
                                             double (&a)[3], double (&jk)[3], double &wmax)
{
    bpl_interact_p<TS>(bpl_partner(L, idx), xi, vi, a, jk, wmax);
}

// Accelerations and jerks of this lane's body from all n-1 partners read
// from the wavefront's LDS slice.  Partner order: the other planets in
// ascending order, then the star (the star lane sums planets 1..n-1), so the
// star's contribution is added last.  Branch-free: the n-2 planet partners
// skip this lane's own index arithmetically and the last partner is peeled.
// ILP unrolls the partner loop fully (the full-register-file kernel class,
// where a wave has its SIMD to itself and needs independent interactions
// in flight); the accumulation order is the same either way.
template <int N, bool TS, bool ILP = false>
__device__ __forceinline__ void bpl_eval(BplLds &L, const int lane, const int b, const int s,
                                         const double (&xi)[3], const double (&vi)[3],
                                         double (&a)[3], double (&jk)[3], double &wmax)
{
    constexpr int S = 64 / N;
    L.xy[lane] = make_double2(xi[0], xi[1]);
    L.zvx[lane] = make_double2(xi[2], vi[0]);
    L.vyvz[lane] = make_double2(vi[1], vi[2]);
    wave_sync();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        a[c] = 0.0;
        jk[c] = 0.0;
    }
    const int own = b == 0 ? 64 : b * S;
    if constexpr (ILP) {
#pragma unroll
        for (int k = 0; k < N - 2; ++k)
            bpl_interact<TS>(L, partner_slot<N>(k, s, own), xi, vi, a, jk, wmax);
    } else {
#pragma unroll FB_BPL_UNROLL
        for (int k = 0; k < N - 2; ++k)
            bpl_interact<TS>(L, partner_slot<N>(k, s, own), xi, vi, a, jk, wmax);
    }
    bpl_interact<TS>(L, (b == 0 ? N - 1 : 0) * S + s, xi, vi, a, jk, wmax);
    wave_sync();
}

template <int N>
__device__ __forceinline__ double sys_max(BplLds &L, int lane, int s, double v)
{
    constexpr int S = 64 / N;
    L.mr[lane].y = v;
    wave_sync();
    double r = L.mr[s].y;
#pragma unroll
    for (int k = 1; k < N; ++k)
        r = fmax(r, L.mr[k * S + s].y);
    wave_sync();
    return r;
}

// Sum over the system's lanes in body order (deterministic).
template <int N>
__device__ __forceinline__ double sys_sum(BplLds &L, int lane, int s, double v)
{
    constexpr int S = 64 / N;
    L.mr[lane].y = v;
    wave_sync();
    double r = L.mr[s].y;
#pragma unroll
    for (int k = 1; k < N; ++k)
        r += L.mr[k * S + s].y;
    wave_sync();
    return r;
}

// OR of the stop-flag bits (1, 2, 4) over the system's lanes (s, s + S, ...)
// from three wave ballots: no LDS round trip.
template <int N>
__device__ __forceinline__ int sys_or_flags(int s, int v)
{
    constexpr int S = 64 / N;
    constexpr unsigned long long kBase = [] {
        unsigned long long m = 0;
        for (int k = 0; k < N; ++k)
            m |= 1ull << (k * S);
        return m;
    }();
    const unsigned long long sm = kBase << s;
    int r = 0;
#pragma unroll
    for (int bit = 1; bit <= 4; bit <<= 1)
        if (__ballot((v & bit) != 0) & sm)
            r |= bit;
    return r;
}

template <int N, bool ILP = false>
__device__ __forceinline__ int bpl_stop_flags(BplLds &L, const int lane, const int b,
                                              const int s, const double mi, const double inv24m0,
                                              const double (&x)[3], const double (&v)[3],
                                              const StepParams &P)
{
    constexpr int S = 64 / N;
    int fl = (finite3(x) && finite3(v)) ? 0 : 1;
    L.xy[lane] = make_double2(x[0], x[1]);
    L.zvx[lane] = make_double2(x[2], 0.0);
    wave_sync();
    const double2 s0 = L.xy[s];
    const double2 s1 = L.zvx[s];
    const double dx = x[0] - s0.x, dy = x[1] - s0.y, dz = x[2] - s1.x;
    const double rb = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
    L.mr[lane].y = rb;
    wave_sync();
    if (b >= 1) {
        if ((P.stop_rules & 2) && rb > P.r_eject)
            fl |= 4;
        if (P.stop_rules & 1) {
            const int own = b * S;
            auto hill = [&](const int k) {
                const int idx = partner_slot<N>(k, s, own);
                const double2 q0 = L.xy[idx];
                const double2 q1 = L.zvx[idx];
                const double ex = x[0] - q0.x, ey = x[1] - q0.y, ez = x[2] - q1.x;
                const double sep2 = fma(ez, ez, fma(ey, ey, ex * ex));
                if (hill_close(sep2, mi, L.mr[idx].x, inv24m0, rb, L.mr[idx].y))
                    fl |= 2;
            };
            if constexpr (ILP) {
#pragma unroll
                for (int k = 0; k < N - 2; ++k)
                    hill(k);
            } else {
#pragma unroll 1
                for (int k = 0; k < N - 2; ++k)
                    hill(k);
            }
        }
    }
    wave_sync();
    return sys_or_flags<N>(s, fl);
}

// Full-register-file variants of the evaluation and of the stop-rule pass,
// for a wave that has its SIMD to itself and so waits out every LDS round
// trip and every dependent latency: the partner slots (pidx) and masses (pm)
// of this lane's body, in evaluation order, are fixed over the run and held
// in registers; all partner reads are issued before the first interaction.
template <int N>
__device__ __forceinline__ int eval_partner(const int k, const int b)
{
    const int skip = b == 0 ? (1 << 20) : b;
    return k < N - 2 ? k + 1 + (k + 1 >= skip ? 1 : 0) : (b == 0 ? N - 1 : 0);
}

template <int N, bool TS>
__device__ __forceinline__ void bpl_eval_regs(BplLds &L, const int lane, const int (&pidx)[N - 1],
                                              const double (&pm)[N - 1], const double (&xi)[3],
                                              const double (&vi)[3], double (&a)[3],
                                              double (&jk)[3], double &wmax)
{
    L.xy[lane] = make_double2(xi[0], xi[1]);
    L.zvx[lane] = make_double2(xi[2], vi[0]);
    L.vyvz[lane] = make_double2(vi[1], vi[2]);
    wave_sync();
    Partner pj[N - 1];
#pragma unroll
    for (int k = 0; k < N - 1; ++k)
        pj[k] = Partner{L.xy[pidx[k]], L.zvx[pidx[k]], L.vyvz[pidx[k]], pm[k]};
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        a[c] = 0.0;
        jk[c] = 0.0;
    }
#pragma unroll
    for (int k = 0; k < N - 1; ++k)
        bpl_interact_p<TS>(pj[k], xi, vi, a, jk, wmax);
    wave_sync();
}

// Stop-rule flags (as bpl_stop_flags) and the system maximum of the step
// rule's w (as sys_max): one exchange of each lane's position and w gives
// the star's position, the partners' positions and every w; a second, of
// the astrocentric distances, the Hill test's partner radii.
template <int N>
__device__ __forceinline__ int bpl_stop_flags_regs(BplLds &L, const int lane, const int b,
                                                   const int s, const int (&pidx)[N - 1],
                                                   const double (&pm)[N - 1], const double mi,
                                                   const double inv24m0, const double (&x)[3],
                                                   const double (&v)[3], const double w,
                                                   double &wsys, const StepParams &P)
{
    int fl = (finite3(x) && finite3(v)) ? 0 : 1;
    L.xy[lane] = make_double2(x[0], x[1]);
    L.zvx[lane] = make_double2(x[2], w);
    wave_sync();
    double2 q0[N - 1], q1[N - 1];
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        q0[k] = L.xy[pidx[k]];
        q1[k] = L.zvx[pidx[k]];
    }
    const double2 s0 = L.xy[s];
    const double2 s1 = L.zvx[s];
    wave_sync();
    // max is exact, so the partners' order gives the body-order result
    wsys = w;
#pragma unroll
    for (int k = 0; k < N - 1; ++k)
        wsys = fmax(wsys, q1[k].y);
    const double dx = x[0] - s0.x, dy = x[1] - s0.y, dz = x[2] - s1.x;
    const double rb = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
    if (P.stop_rules & 1) {
        // the partners' astrocentric distances: a second exchange is
        // shorter than computing N - 2 more square roots per lane
        double rp[N - 1];
        L.mr[lane].y = rb;
        wave_sync();
#pragma unroll
        for (int k = 0; k < N - 2; ++k)
            rp[k] = L.mr[pidx[k]].y;
        wave_sync();
        if (b >= 1) {
#pragma unroll
            for (int k = 0; k < N - 2; ++k) {
                const double ex = x[0] - q0[k].x, ey = x[1] - q0[k].y, ez = x[2] - q1[k].x;
                const double sep2 = fma(ez, ez, fma(ey, ey, ex * ex));
                if (hill_close(sep2, mi, pm[k], inv24m0, rb, rp[k]))
                    fl |= 2;
            }
        }
    }
    if (b >= 1 && (P.stop_rules & 2) && rb > P.r_eject)
        fl |= 4;
    return sys_or_flags<N>(s, fl);
}

// Integrate one tile (floor(64/N) systems) with one body per lane for at
// most P.quantum steps.  Every lane of the wavefront executes the same
// control flow (the LDS exchanges need it); lanes of finished, padding or
// absent systems compute but never commit.  Returns, on the star lane of each
// present system, whether that system is still active.
template <int N, bool ADV, bool WIDE>
__device__ __forceinline__ bool bpl_run(const Bucket &B, const int first, const int count, const int *list,
                        const StepParams &P, int &slot_out)
{
    constexpr int S = 64 / N;
    BplLds &L = *reinterpret_cast<BplLds *>(wave_lds_base<sizeof(BplLds), WIDE>());
    const int lane = threadIdx.x & 63;
    const int braw = lane / S;
    const int b = braw < N ? braw : N - 1;
    const int s = lane - braw * S;
    const bool valid = braw < N && s < count;
    int slot = 0;
    if (valid)
        slot = list ? list[first + s] : first + s;
    slot_out = slot;
    const size_t pitch = B.pitch;
    double mi = 0.0, x[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0};
    double a0[3] = {0.0, 0.0, 0.0}, j0[3] = {0.0, 0.0, 0.0};
    Clock c{};
    c.status = ST_DONE;
    if (valid) {
        mi = B.st[(R_M * N + b) * pitch + slot];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            x[cc] = B.st[((R_X + cc) * N + b) * pitch + slot];
            v[cc] = B.st[((R_V + cc) * N + b) * pitch + slot];
            a0[cc] = B.st[((R_A + cc) * N + b) * pitch + slot];
            j0[cc] = B.st[((R_J + cc) * N + b) * pitch + slot];
        }
        c = load_clock(B, slot);
    }
    L.mr[lane].x = mi;
    wave_sync();
    // Hill-test scale of the system's star, fixed over the run.
    const double inv24m0 = ADV ? 1.0 / (24.0 * L.mr[s].x) : 0.0;
    // The full-register-file class keeps the partner tables in registers.
    constexpr bool REGS = WIDE && N <= 8;
    int pidx[N - 1];
    double pm[N - 1];
#pragma unroll
    for (int k = 0; k < N - 1; ++k) {
        pidx[k] = REGS ? eval_partner<N>(k, b) * S + s : 0;
        pm[k] = REGS ? L.mr[pidx[k]].x : 0.0;
    }
    for (int q = 0; q < P.quantum; ++q) {
        double h = 0.0;
        bool last = false;
        bool act;
        if constexpr (ADV && REGS)   // invalid lanes hold an inactive clock
            act = P.adaptive ? plan_step_adaptive(c, P, h, last) : valid && plan_step(c, P, h, last);
        else
            act = valid && plan_step(c, P, h, last);
        if (!__any(act))
            break;
        const Coef k = make_coef(h);
        double xc[3], vc[3], bx[3], bv[3], ak[3], jk[3];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            predict_comp(k, x[cc], v[cc], a0[cc], j0[cc], xc[cc], vc[cc], bx[cc], bv[cc]);
        double w = 0.0;
        if constexpr (REGS)
            bpl_eval_regs<N, false>(L, lane, pidx, pm, xc, vc, ak, jk, w);
        else
            bpl_eval<N, false, WIDE>(L, lane, b, s, xc, vc, ak, jk, w);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            correct_comp(k, bx[cc], bv[cc], ak[cc], jk[cc], xc[cc], vc[cc]);
        if constexpr (REGS)
            bpl_eval_regs<N, ADV>(L, lane, pidx, pm, xc, vc, ak, jk, w);
        else
            bpl_eval<N, ADV, WIDE>(L, lane, b, s, xc, vc, ak, jk, w);
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
            correct_comp(k, bx[cc], bv[cc], ak[cc], jk[cc], xc[cc], vc[cc]);
        if constexpr (ADV && REGS) {
            // commit, then one exchange for the step rule's maximum and the
            // stop rules (same values and order of decisions as below)
            double dtp = 0.0;
            if (P.adaptive == 2) {
                const double aa = fma(ak[2], ak[2], fma(ak[1], ak[1], ak[0] * ak[0]));
                const double jj = fma(jk[2], jk[2], fma(jk[1], jk[1], jk[0] * jk[0]));
                dtp = P.eta * rsqrt_nr(sys_sum<N>(L, lane, s, jj / aa));
            }
            if (act) {
#pragma unroll
                for (int cc = 0; cc < 3; ++cc) {
                    x[cc] = xc[cc];
                    v[cc] = vc[cc];
                    a0[cc] = ak[cc];
                    j0[cc] = jk[cc];
                }
            }
            double wsys = 0.0;
            const int fl = bpl_stop_flags_regs<N>(L, lane, b, s, pidx, pm, mi, inv24m0, x, v, w,
                                                  wsys, P);
            if (P.adaptive == 1)
                dtp = P.eta * rsqrt_nr(wsys);
            if (P.adaptive) {
                finish_step_adaptive(c, act, last, h, dtp, fl);
            } else if (act) {
                finish_step(c, P, last, h, dtp);
                if (fl)
                    c.status = status_of_flags(fl);
            }
            continue;
        }
        double dtp = 0.0;
        if (ADV && P.adaptive == 1)
            dtp = P.eta * rsqrt_nr(sys_max<N>(L, lane, s, w));
        if (ADV && P.adaptive == 2) {
            const double aa = fma(ak[2], ak[2], fma(ak[1], ak[1], ak[0] * ak[0]));
            const double jj = fma(jk[2], jk[2], fma(jk[1], jk[1], jk[0] * jk[0]));
            dtp = P.eta * rsqrt_nr(sys_sum<N>(L, lane, s, jj / aa));
        }
        if (act) {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                x[cc] = xc[cc];
                v[cc] = vc[cc];
                a0[cc] = ak[cc];
                j0[cc] = jk[cc];
            }
            finish_step(c, P, last, h, dtp);
        }
        if (ADV) {
            const int fl = bpl_stop_flags<N, WIDE>(L, lane, b, s, mi, inv24m0, x, v, P);
            if (act && fl)
                c.status = status_of_flags(fl);
        }
    }
    if (!ADV) {
        const int fl = sys_or_flags<N>(s, (finite3(x) && finite3(v)) ? 0 : 1);
        if (valid && fl)
            c.status = ST_NONFINITE;
    }
    if (valid) {
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            B.st[((R_X + cc) * N + b) * pitch + slot] = x[cc];
            B.st[((R_V + cc) * N + b) * pitch + slot] = v[cc];
            B.st[((R_A + cc) * N + b) * pitch + slot] = a0[cc];
            B.st[((R_J + cc) * N + b) * pitch + slot] = j0[cc];
        }
        if (b == 0)
            store_clock(B, slot, c);
    }
    return valid && b == 0 && braw == 0 && c.status == ST_ACTIVE;
}

// ---------------------------------------------------------------------------
// kernels: plain schedule (one launch per homogeneous bucket)
// ---------------------------------------------------------------------------
// The system-per-lane run of 9 and 10 bodies as a separately compiled
// function: inlined into the kernel, the register allocator spilled 92 and
// 476 bytes per lane to scratch memory; as a callee it spills to AGPRs only.
template <int N, bool ADV>
__device__ __noinline__ void spl_plain_call(const Bucket &B, const int slot, const StepParams &P)
{
    spl_run<N, ADV, false>(B, slot, uniform_params(P));
}

template <int N, bool ADV>
__global__ __launch_bounds__(256) void k_plain_spl(Bucket B, StepParams P)
{
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= B.count)
        return;
    if constexpr (N >= 9)
        spl_plain_call<N, ADV>(B, slot, P);
    else
        spl_run<N, ADV, false>(B, slot, P);
}

template <int N, bool ADV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FB_BPL_WAVES)))
void k_plain_bpl(Bucket B, StepParams P)
{
    constexpr int S = 64 / N;
    const int wave = threadIdx.x >> 6;
    const int tile = blockIdx.x * (blockDim.x >> 6) + wave;
    const int first = tile * S;
    if (first >= B.count)
        return;
    const int count = min(S, B.count - first);
    int slot;
    bpl_run<N, ADV, false>(B, first, count, nullptr, P, slot);
}

// ---------------------------------------------------------------------------
// kernel: persistent schedule (one fused launch over every bucket)
// ---------------------------------------------------------------------------

// Append the systems flagged by `keep` to bucket `bk`'s survivor list
// (wave-aggregated: one atomic per wavefront).
__device__ __forceinline__ void append_survivors(const ActiveLists &AL, int bk, bool keep,
                                                 int slot)
{
    const int lane = threadIdx.x & 63;
    const unsigned long long mask = __ballot(keep);
    if (mask == 0ull)
        return;
    const int cnt = __popcll(mask);
    int base = 0;
    if (lane == 0)
        base = atomicAdd(&AL.next_count[bk], cnt);
    base = __builtin_amdgcn_readfirstlane(base);
    const int pre = __popcll(mask & ((1ull << lane) - 1ull));
    if (keep)
        AL.next[AL.base[bk] + base + pre] = slot;
}

// The tile functions are separately compiled, so their reference arguments
// arrive as generic pointers; the step loop works on a register copy of the
// step parameters (read once), not on memory it would reload after every LDS
// exchange.  The copy is made wave-uniform (scalar registers), so the tests
// on it are scalar branches rather than exec-mask changes.
template <int N, bool ADV>
__device__ __noinline__ bool spl_tile(const Bucket &B, const Tile &T, const int *list,
                                      const StepParams &P, int &slot)
{
    const StepParams Pr = uniform_params(P);
    const int lane = threadIdx.x & 63;
    slot = 0;
    if (lane >= T.count)
        return false;
    slot = list ? list[T.first + lane] : T.first + lane;
    spl_run<N, ADV, true>(B, slot, Pr);
    return B.status[slot] == ST_ACTIVE;
}

// CLS only separates the instances used by the two fused-kernel classes, so
// each is compiled under its own kernel's register budget.
template <int N, bool ADV, bool CLS>
__device__ __noinline__ bool bpl_tile(const Bucket &B, const Tile &T, const int *list,
                                      const StepParams &P, int &slot)
{
    const StepParams Pr = uniform_params(P);
    return bpl_run<N, ADV, CLS>(B, T.first, T.count, list, Pr, slot);
}

// Tile dispatch.  The body-per-lane class (SPLC false) keeps the fused
// kernel at <= 168 VGPRs (3 waves per SIMD) and runs every tile body-per-
// lane; the system-per-lane class gives the kernel the full register file
// (1 wave per SIMD) and runs system-per-lane tiles up to n = 10 (n = 8 with
// adaptive steps / stop rules), body-per-lane beyond.
template <bool ADV, bool SPLC>
__device__ __forceinline__ bool run_tile(const Bucket &B, const Tile &T, const int *list,
                                         const StepParams &P, int &slot)
{
    const int map = T.kind >> 5;
    const int n = T.kind & 31;
    if (map == MAP_SPL) {
        if constexpr (SPLC) {
            switch (n) {
            case 2: return spl_tile<2, ADV>(B, T, list, P, slot);
            case 3: return spl_tile<3, ADV>(B, T, list, P, slot);
            case 4: return spl_tile<4, ADV>(B, T, list, P, slot);
            case 5: return spl_tile<5, ADV>(B, T, list, P, slot);
            case 6: return spl_tile<6, ADV>(B, T, list, P, slot);
            case 7: return spl_tile<7, ADV>(B, T, list, P, slot);
            case 8: return spl_tile<8, ADV>(B, T, list, P, slot);
            default: break;
            }
            if constexpr (!ADV) {
                switch (n) {
                case 9: return spl_tile<9, false>(B, T, list, P, slot);
                case 10: return spl_tile<10, false>(B, T, list, P, slot);
                default: break;
                }
            }
        }
    }
    switch (n) {
#define FB_BPL_CASE(NN) case NN: return bpl_tile<NN, ADV, SPLC>(B, T, list, P, slot);
        FB_BPL_CASE(2) FB_BPL_CASE(3) FB_BPL_CASE(4) FB_BPL_CASE(5) FB_BPL_CASE(6)
        FB_BPL_CASE(7) FB_BPL_CASE(8) FB_BPL_CASE(9) FB_BPL_CASE(10) FB_BPL_CASE(11)
        FB_BPL_CASE(12) FB_BPL_CASE(13) FB_BPL_CASE(14) FB_BPL_CASE(15) FB_BPL_CASE(16)
#undef FB_BPL_CASE
    default: return false;
    }
}

template <bool ADV, bool COMPACT, bool SPLC>
__device__ __forceinline__ void persistent_body(const Bucket *__restrict__ buckets,
                                                const Tile *__restrict__ tiles,
                                                const int *__restrict__ ntiles_p,
                                                int *__restrict__ head, const int *lists,
                                                const StepParams &P, const ActiveLists &AL)
{
    const int ntiles = *ntiles_p;
    const int lane = threadIdx.x & 63;
    // Each wave's first tile is its own index; the rest come from the queue
    // (past the first round).  Workgroups are dispatched across the CUs in
    // index order, so when the tiles are fewer than the resident waves (the
    // population has thinned) they land one per SIMD rather than wherever
    // the queue's atomics happen to be served first.
    const int nwaves = (int)(gridDim.x * (blockDim.x >> 6));
    int first = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6));
    for (;;) {
        int t = 0;
        if (first >= 0) {
            t = first;
            first = -1;
        } else {
            if (lane == 0)
                t = nwaves + atomicAdd(head, 1);
            t = __builtin_amdgcn_readfirstlane(t);
        }
        if (t >= ntiles)
            break;
        const Tile T = tiles[t];
        const Bucket B = buckets[T.bucket];
        int slot = 0;
        const bool keep = run_tile<ADV, SPLC>(B, T, lists, P, slot);
        if (COMPACT)
            append_survivors(AL, T.bucket, keep, slot);
    }
}

template <bool ADV, bool COMPACT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FB_BPL_WAVES)))
void k_persistent(const Bucket *__restrict__ buckets, const Tile *__restrict__ tiles,
                  const int *__restrict__ ntiles_p, int *__restrict__ head, const int *lists,
                  StepParams P, ActiveLists AL)
{
    persistent_body<ADV, COMPACT, false>(buckets, tiles, ntiles_p, head, lists, P, AL);
}

template <bool ADV, bool COMPACT>
__global__ __launch_bounds__(256) void k_persistent_spl(const Bucket *__restrict__ buckets,
                                                        const Tile *__restrict__ tiles,
                                                        const int *__restrict__ ntiles_p,
                                                        int *__restrict__ head,
                                                        const int *lists, StepParams P,
                                                        ActiveLists AL)
{
    persistent_body<ADV, COMPACT, true>(buckets, tiles, ntiles_p, head, lists, P, AL);
}

// Tiles for the next quantum from the survivor counts (one workgroup):
// buckets in the given order (longest work first), tiles of each bucket in
// list order; resets the queue head and the other list's counts.
__global__ void k_build_tiles(const Bucket *__restrict__ buckets, int nb,
                              const int *__restrict__ order, const int *__restrict__ mapping,
                              ActiveLists AL, Tile *__restrict__ tiles, int *ntiles,
                              int *head)
{
    __shared__ int start[kMaxBodies + 2];
    __shared__ int cap[kMaxBodies + 2];
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < nb; ++i) {
            const int bk = order[i];
            const int n = buckets[bk].n;
            const int c = (mapping[bk] == MAP_SPL) ? 64 : 64 / n;
            cap[i] = c;
            start[i] = acc;
            acc += (AL.cur_count[bk] + c - 1) / c;
        }
        start[nb] = acc;
        *ntiles = acc;
        *head = 0;
    }
    __syncthreads();
    for (int i = 0; i < nb; ++i) {
        const int bk = order[i];
        const int n = buckets[bk].n;
        const int cnt = AL.cur_count[bk];
        const int c = cap[i];
        for (int t = threadIdx.x; t < start[i + 1] - start[i]; t += blockDim.x) {
            Tile T;
            T.bucket = bk;
            T.first = AL.base[bk] + t * c;
            T.count = min(c, cnt - t * c);
            T.kind = mapping[bk] * 32 + n;
            tiles[start[i] + t] = T;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nb; i += blockDim.x)
        AL.next_count[order[i]] = 0;
}

__global__ void k_fill_int(int *p, int n, int value)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        p[i] = value;
}

// ---------------------------------------------------------------------------
// set-up, run control, layout and diagnostics kernels (one thread per slot)
// ---------------------------------------------------------------------------

// AoS (caller order) -> bucket SoA; validates the inputs.
__global__ void k_pack(Bucket B, const double *__restrict__ mass, const double *__restrict__ pos,
                       const double *__restrict__ vel, const double *__restrict__ t0,
                       const long long *__restrict__ orig_off, int *bad, int limit)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= limit)
        return;
    const size_t pitch = B.pitch;
    const int n = B.n;
    if (s >= B.count) {   // padding slots: inert, finished
        B.status[s] = ST_DONE;
        B.t[s] = 0.0;
        B.steps[s] = 0;
        return;
    }
    const int o = B.orig[s];
    const long long base = orig_off[o];
    bool ok = true;
    for (int b = 0; b < n; ++b) {
        const double m = mass[base + b];
        ok = ok && __builtin_isfinite(m) && m >= 0.0;
        B.st[(R_M * n + b) * pitch + s] = m;
        for (int c = 0; c < 3; ++c) {
            const double xv = pos[3 * (base + b) + c];
            const double vv = vel[3 * (base + b) + c];
            ok = ok && __builtin_isfinite(xv) && __builtin_isfinite(vv);
            B.st[((R_X + c) * n + b) * pitch + s] = xv;
            B.st[((R_V + c) * n + b) * pitch + s] = vv;
        }
    }
    const double tt = t0 ? t0[o] : 0.0;
    ok = ok && __builtin_isfinite(tt);
    B.t[s] = tt;
    B.t0run[s] = tt;
    B.t_end[s] = tt;
    B.dt[s] = 0.0;
    B.dtn[s] = 0.0;
    B.krun[s] = 0;
    B.nfull[s] = 0;
    B.steps[s] = 0;
    B.status[s] = ST_DONE;
    if (!ok)
        atomicOr(bad, 1);
}

template <int N>
__device__ __forceinline__ void load_xv(const Bucket &B, int s, double (&m)[N], double (&x)[N][3],
                                        double (&v)[N][3])
{
    const size_t pitch = B.pitch;
#pragma unroll
    for (int b = 0; b < N; ++b) {
        m[b] = B.st[(R_M * N + b) * pitch + s];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[b][c] = B.st[((R_X + c) * N + b) * pitch + s];
            v[b][c] = B.st[((R_V + c) * N + b) * pitch + s];
        }
    }
}

// Algorithm 1's "prepare": (a0, j0) at the initial state.
template <int N>
__global__ void k_prepare(Bucket B)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B.count)
        return;
    double m[N], x[N][3], v[N][3], a[N][3], jk[N][3];
    load_xv<N>(B, s, m, x, v);
    double w = 0.0;
    spl_accjerk<N, false>(m, x, v, a, jk, w);
    const size_t pitch = B.pitch;
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            B.st[((R_A + c) * N + b) * pitch + s] = a[b][c];
            B.st[((R_J + c) * N + b) * pitch + s] = jk[b][c];
        }
}

// Start a run.  fixed_steps: exactly n_steps steps of dt.  Otherwise to
// t_end, with fixed dt or (adaptive) the carried step, proposing one from
// the current state when none is carried yet.  Systems stopped by a rule
// keep their status.
// The clock part of a run's start for slot s; true when an adaptive step
// (rule 1 or 2) must still be proposed from the system's state.
__device__ __forceinline__ bool begin_run_clock(const Bucket &B, const int s, int fixed_steps,
                                                long long n_steps, double t_end, double dt,
                                                int adaptive)
{
    const int st = B.status[s];
    if (st != ST_ACTIVE && st != ST_DONE && st != ST_MAXSTEPS)
        return false;
    const double t = B.t[s];
    B.t0run[s] = t;
    B.krun[s] = 0;
    if (fixed_steps) {
        B.dt[s] = dt;
        B.nfull[s] = n_steps;
        B.t_end[s] = fma((double)n_steps, dt, t);
        B.status[s] = n_steps > 0 ? ST_ACTIVE : ST_DONE;
        return false;
    }
    B.t_end[s] = t_end;
    if (adaptive == 3) {   // Runge-Kutta Cash-Karp: dt is the first trial step
        B.nfull[s] = 0;
        B.dt[s] = 0.0;
        B.dtn[s] = dt;
        B.status[s] = t < t_end ? ST_ACTIVE : ST_DONE;
        return false;
    }
    if (adaptive) {
        B.nfull[s] = 0;
        B.dt[s] = 0.0;
        B.status[s] = t < t_end ? ST_ACTIVE : ST_DONE;
        // Eq. 5's step depends only on the stored (a0, j0), so it is always
        // recomputed (identical to the carried value); the pairwise rule's
        // carried step comes from the last evaluation's state and is kept.
        return adaptive == 2 || !(B.dtn[s] > 0.0);
    }
    B.dt[s] = dt;
    const double span = (t_end - t) / dt;
    long long nf = span > 0.0 ? (long long)floor(span) : 0;
    while (nf > 0 && (fma((double)nf, dt, t) - t_end) * dt > 0.0)
        --nf;
    B.nfull[s] = nf;
    B.status[s] = (t_end - t) * dt > 0.0 ? ST_ACTIVE : ST_DONE;
    return false;
}

template <int N>
__global__ void k_begin_run(Bucket B, int fixed_steps, long long n_steps, double t_end,
                            double dt, int adaptive, double eta)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B.count)
        return;
    if (!begin_run_clock(B, s, fixed_steps, n_steps, t_end, dt, adaptive))
        return;
    double m[N], x[N][3], v[N][3], a[N][3], jk[N][3];
    load_xv<N>(B, s, m, x, v);
    if (adaptive == 2) {
        const size_t pitch = B.pitch;
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                a[b][c] = B.st[((R_A + c) * N + b) * pitch + s];
                jk[b][c] = B.st[((R_J + c) * N + b) * pitch + s];
            }
        B.dtn[s] = paper_dt<N>(a, jk, eta);
    } else {
        double w = 0.0;
        spl_accjerk<N, true>(m, x, v, a, jk, w);
        B.dtn[s] = eta * rsqrt_nr(w);
    }
}


// bucket SoA -> AoS rows in caller order (any output may be null).
__global__ void k_unpack(Bucket B, const long long *__restrict__ orig_off, double *pos,
                         double *vel, double *acc, double *jerk, double *t, int *status,
                         long long *steps, double *dtn)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B.count)
        return;
    const size_t pitch = B.pitch;
    const int n = B.n;
    const int o = B.orig[s];
    const long long base = orig_off[o];
    for (int b = 0; b < n; ++b)
        for (int c = 0; c < 3; ++c) {
            const size_t row = 3 * (base + b) + c;
            if (pos) pos[row] = B.st[((R_X + c) * n + b) * pitch + s];
            if (vel) vel[row] = B.st[((R_V + c) * n + b) * pitch + s];
            if (acc) acc[row] = B.st[((R_A + c) * n + b) * pitch + s];
            if (jerk) jerk[row] = B.st[((R_J + c) * n + b) * pitch + s];
        }
    if (t) t[o] = B.t[s];
    if (status) status[o] = B.status[s];
    if (steps) steps[o] = B.steps[s];
    if (dtn) dtn[o] = B.dtn[s];
}

template <int N>
__device__ __forceinline__ void from_mvs(const double (&m)[N], double (&x)[N][3], double (&v)[N][3]);

// Energy (Eq. 6, each pair once) and angular momentum about the origin of
// one system.
template <int N>
__device__ __forceinline__ void sys_energy(const double (&m)[N], const double (&x)[N][3],
                                          const double (&v)[N][3], double &energy,
                                          double (&L)[3])
{
    double kin = 0.0, pot = 0.0, L0 = 0.0, L1 = 0.0, L2 = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        kin += 0.5 * m[i] * fma(v[i][2], v[i][2], fma(v[i][1], v[i][1], v[i][0] * v[i][0]));
        L0 += m[i] * (x[i][1] * v[i][2] - x[i][2] * v[i][1]);
        L1 += m[i] * (x[i][2] * v[i][0] - x[i][0] * v[i][2]);
        L2 += m[i] * (x[i][0] * v[i][1] - x[i][1] * v[i][0]);
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = i + 1; j < N; ++j) {
            const double dx = x[i][0] - x[j][0], dy = x[i][1] - x[j][1], dz = x[i][2] - x[j][2];
            pot += m[i] * m[j] / sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
        }
    energy = kin - pot;
    L[0] = L0;
    L[1] = L1;
    L[2] = L2;
}

// Energy and angular momentum of every system of a bucket in inertial form
// or (MVS) in MVS form, converted first.
template <int N, bool MVS>
__global__ void k_diag(Bucket B, double *energy, double *angmom)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B.count)
        return;
    double m[N], x[N][3], v[N][3];
    load_xv<N>(B, s, m, x, v);
    if (MVS)
        from_mvs<N>(m, x, v);
    double E, L[3];
    sys_energy<N>(m, x, v, E, L);
    const int o = B.orig[s];
    if (energy)
        energy[o] = E;
    if (angmom) {
        angmom[3 * o + 0] = L[0];
        angmom[3 * o + 1] = L[1];
        angmom[3 * o + 2] = L[2];
    }
}

// Monitor record k of every system of a bucket (Section 4.3's logging, with
// Section 4.4's data reduction), into the caller's log buffer:
//   kind 0 (state):  system o's block starts at max_records (o + 6 off[o])
//                    doubles; record k holds t, then pos [n][3], vel [n][3];
//   kind 1 (RV):     [o][k][2] = t and the star's velocity relative to the
//                    system's centre of mass along the unit line of sight l;
//   kind 2 (energy): [o][k][5] = t, E, L.
template <int N>
__global__ void k_log(Bucket B, const long long *__restrict__ orig_off, int kind, double lx,
                      double ly, double lz, int k, int max_records, double *out)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B.count)
        return;
    double m[N], x[N][3], v[N][3];
    load_xv<N>(B, s, m, x, v);
    const int o = B.orig[s];
    const double t = B.t[s];
    if (kind == 1) {
        double M = 0.0, p0 = 0.0, p1 = 0.0, p2 = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            M += m[i];
            p0 = fma(m[i], v[i][0], p0);
            p1 = fma(m[i], v[i][1], p1);
            p2 = fma(m[i], v[i][2], p2);
        }
        const double rv = fma(v[0][2] - p2 / M, lz, fma(v[0][1] - p1 / M, ly, (v[0][0] - p0 / M) * lx));
        double *r = out + ((size_t)o * max_records + k) * 2;
        r[0] = t;
        r[1] = rv;
    } else if (kind == 2) {
        double E, L[3];
        sys_energy<N>(m, x, v, E, L);
        double *r = out + ((size_t)o * max_records + k) * 5;
        r[0] = t;
        r[1] = E;
        r[2] = L[0];
        r[3] = L[1];
        r[4] = L[2];
    } else {
        double *r = out + (size_t)max_records * ((size_t)o + 6 * (size_t)orig_off[o]) +
                    (size_t)k * (1 + 6 * N);
        r[0] = t;
#pragma unroll
        for (int b = 0; b < N; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                r[1 + 3 * b + c] = x[b][c];
                r[1 + 3 * N + 3 * b + c] = v[b][c];
            }
    }
}

__global__ void k_count_active(Bucket B, int *count)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    const bool act = s < B.count && B.status[s] == ST_ACTIVE;
    const unsigned long long mask = __ballot(act);
    if ((threadIdx.x & 63) == 0 && mask)
        atomicAdd(count, __popcll(mask));
}

// ---------------------------------------------------------------------------
// mixed-variable symplectic (MVS) integrator, Sections 2.2.3 and 4.3.3
// ---------------------------------------------------------------------------
// The paper's five sub-steps (Cartesian drift half step, kick half step,
// Keplerian drift step, kick half step, Cartesian drift half step) are the
// democratic heliocentric splitting (Duncan, Levison & Lee 1998): planets
// move on Kepler orbits about the star with mu = m0 in heliocentric
// positions Q_i = x_i - x_0 and barycentric velocities V_i; kicks apply the
// planet-planet forces only; the drift moves every Q_i by the star's reflex
// motion, dt sum_j m_j V_j / m0, and the centre of mass by dt Vc.
//
// A bucket in MVS form keeps body 0's x and v rows for the centre of mass X
// and its velocity Vc, body i's rows for Q_i and V_i, and the a rows for the
// planet-planet accelerations at Q, which the next step's first kick reuses:
// the drifts move all Q_i together, so the separations do not change.

// (r, v) advanced by dt on its Kepler orbit about mu.  The change x of the
// eccentric anomaly solves Kepler's equation in difference form,
//   n dt = x - (1 - r0/a) sin x + (r.v / sqrt(mu a)) (1 - cos x),
// by Newton iteration from x = n dt; Lagrange's f and g functions give the
// new state.  The caller has checked 1/a > 0.  Returns false if the
// iteration does not converge in kMvsNewtonMax steps.
constexpr int kMvsNewtonMax = 50;

__device__ __forceinline__ bool kepler_drift(const double mu, double (&r)[3], double (&v)[3],
                                             const double dt)
{
    const double r2 = fma(r[2], r[2], fma(r[1], r[1], r[0] * r[0]));
    const double v2 = fma(v[2], v[2], fma(v[1], v[1], v[0] * v[0]));
    const double rv = fma(r[2], v[2], fma(r[1], v[1], r[0] * v[0]));
    const double r0 = sqrt(r2);
    const double alpha = 2.0 / r0 - v2 / mu;
    const double a = 1.0 / alpha;
    const double sqmua = sqrt(mu * a);
    const double nmot = sqmua * alpha * alpha;   // sqrt(mu / a^3)
    const double ec = 1.0 - r0 * alpha;
    const double es = rv / sqmua;
    const double M = nmot * dt;
    double x = M, s = 0.0, c = 1.0;
    bool ok = false;
    for (int it = 0; it < kMvsNewtonMax; ++it) {
        sincos(x, &s, &c);
        const double F = fma(-ec, s, x) + fma(es, 1.0 - c, -M);
        const double dF = fma(es, s, fma(-ec, c, 1.0));
        const double dx = F / dF;
        x -= dx;
        if (fabs(dx) <= 1e-15 * (1.0 + fabs(x))) {
            ok = true;
            break;
        }
    }
    if (!ok)
        return false;
    sincos(x, &s, &c);
    const double omc = 1.0 - c;
    const double f = fma(-a / r0, omc, 1.0);
    const double g = dt - (x - s) / nmot;
    const double rn = a * fma(es, s, fma(-ec, c, 1.0));
    const double fd = -sqmua * s / (rn * r0);
    const double gd = fma(-a / rn, omc, 1.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double rk = r[k], vk = v[k];
        r[k] = fma(f, rk, g * vk);
        v[k] = fma(fd, rk, gd * vk);
    }
    return true;
}

// Planet-planet accelerations at heliocentric positions Q[1..N-1].
template <int N>
__device__ __forceinline__ void mvs_acc(const double (&m)[N], const double (&Q)[N][3],
                                        double (&acc)[N][3])
{
#pragma unroll
    for (int i = 1; i < N; ++i)
        acc[i][0] = acc[i][1] = acc[i][2] = 0.0;
#pragma unroll
    for (int i = 1; i < N; ++i)
#pragma unroll
        for (int j = i + 1; j < N; ++j) {
            const double d0 = Q[j][0] - Q[i][0], d1 = Q[j][1] - Q[i][1], d2 = Q[j][2] - Q[i][2];
            const double s = rsqrt_nr(fma(d2, d2, fma(d1, d1, d0 * d0)));
            const double s3 = s * s * s;
            const double mj = m[j] * s3, mi = m[i] * s3;
            acc[i][0] = fma(mj, d0, acc[i][0]);
            acc[i][1] = fma(mj, d1, acc[i][1]);
            acc[i][2] = fma(mj, d2, acc[i][2]);
            acc[j][0] = fma(-mi, d0, acc[j][0]);
            acc[j][1] = fma(-mi, d1, acc[j][1]);
            acc[j][2] = fma(-mi, d2, acc[j][2]);
        }
}

// Drift of every Q_i by h sum_j m_j V_j / m0 and of X by h Vc (body 0's rows).
template <int N>
__device__ __forceinline__ void mvs_drift(const double (&m)[N], double (&Q)[N][3],
                                          const double (&V)[N][3], const double inv_m0,
                                          const double h)
{
    double P[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int i = 1; i < N; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            P[c] = fma(m[i], V[i][c], P[c]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double dq = h * P[c] * inv_m0;
#pragma unroll
        for (int i = 1; i < N; ++i)
            Q[i][c] += dq;
        Q[0][c] = fma(h, V[0][c], Q[0][c]);
    }
}

template <int N>
__device__ __forceinline__ void mvs_kick(double (&V)[N][3], const double (&acc)[N][3], const double h)
{
#pragma unroll
    for (int i = 1; i < N; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            V[i][c] = fma(h, acc[i][c], V[i][c]);
}

// One MVS step of h.  Returns ST_ACTIVE, or ST_UNBOUND when a planet's
// heliocentric orbit is not bound (the half drift and kick are undone, so
// the state is the step's start up to rounding) or Kepler's equation does not
// converge (state of the planets drifted so far).
template <int N>
__device__ __forceinline__ int mvs_step(const double (&m)[N], double (&Q)[N][3], double (&V)[N][3],
                                        double (&acc)[N][3], const double inv_m0, const double h)
{
    const double hh = 0.5 * h;
    mvs_drift<N>(m, Q, V, inv_m0, hh);
    mvs_kick<N>(V, acc, hh);
    bool bound = true;
#pragma unroll
    for (int i = 1; i < N; ++i) {
        const double r2 = fma(Q[i][2], Q[i][2], fma(Q[i][1], Q[i][1], Q[i][0] * Q[i][0]));
        const double v2 = fma(V[i][2], V[i][2], fma(V[i][1], V[i][1], V[i][0] * V[i][0]));
        bound = bound && (2.0 / sqrt(r2) - v2 / m[0] > 0.0);
    }
    if (!bound) {
        mvs_kick<N>(V, acc, -hh);
        mvs_drift<N>(m, Q, V, inv_m0, -hh);
        return ST_UNBOUND;
    }
#pragma unroll
    for (int i = 1; i < N; ++i)
        if (!kepler_drift(m[0], Q[i], V[i], h))
            return ST_UNBOUND;
    mvs_acc<N>(m, Q, acc);
    mvs_kick<N>(V, acc, hh);
    mvs_drift<N>(m, Q, V, inv_m0, hh);
    return ST_ACTIVE;
}

template <int N>
__device__ __forceinline__ void load_rows(const Bucket &B, int s, double (&m)[N], double (&x)[N][3],
                                          double (&v)[N][3], double (&a)[N][3], bool with_a)
{
    const size_t pitch = B.pitch;
#pragma unroll
    for (int b = 0; b < N; ++b) {
        m[b] = B.st[(R_M * N + b) * pitch + s];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[b][c] = B.st[((R_X + c) * N + b) * pitch + s];
            v[b][c] = B.st[((R_V + c) * N + b) * pitch + s];
            a[b][c] = with_a ? B.st[((R_A + c) * N + b) * pitch + s] : 0.0;
        }
    }
}

template <int N>
__device__ __forceinline__ void store_rows(const Bucket &B, int s, const double (&x)[N][3],
                                           const double (&v)[N][3], const double (&a)[N][3],
                                           bool with_a)
{
    const size_t pitch = B.pitch;
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            B.st[((R_X + c) * N + b) * pitch + s] = x[b][c];
            B.st[((R_V + c) * N + b) * pitch + s] = v[b][c];
            if (with_a)
                B.st[((R_A + c) * N + b) * pitch + s] = a[b][c];
        }
}

// Inertial (x, v) -> MVS form in place: X, Vc in row 0, Q_i = x_i - x_0,
// V_i = v_i - Vc, and the planet-planet accelerations at Q.
template <int N>
__device__ __forceinline__ void to_mvs(const double (&m)[N], double (&x)[N][3], double (&v)[N][3])
{
    double M = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
        M += m[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double sx = 0.0, sv = 0.0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
            sx = fma(m[i], x[i][c], sx);
            sv = fma(m[i], v[i][c], sv);
        }
        const double X = sx / M, Vc = sv / M, x0 = x[0][c];
#pragma unroll
        for (int i = 1; i < N; ++i) {
            x[i][c] -= x0;
            v[i][c] -= Vc;
        }
        x[0][c] = X;
        v[0][c] = Vc;
    }
}

// MVS form -> inertial in place: x_0 = X - sum m_i Q_i / M, x_i = x_0 + Q_i,
// v_0 = Vc - sum m_i V_i / m0, v_i = Vc + V_i.
template <int N>
__device__ __forceinline__ void from_mvs(const double (&m)[N], double (&x)[N][3], double (&v)[N][3])
{
    double M = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i)
        M += m[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double sq = 0.0, sp = 0.0;
#pragma unroll
        for (int i = 1; i < N; ++i) {
            sq = fma(m[i], x[i][c], sq);
            sp = fma(m[i], v[i][c], sp);
        }
        const double x0 = x[0][c] - sq / M, Vc = v[0][c];
        x[0][c] = x0;
        v[0][c] = Vc - sp / m[0];
#pragma unroll
        for (int i = 1; i < N; ++i) {
            x[i][c] += x0;
            v[i][c] += Vc;
        }
    }
}

template <int N>
__global__ __launch_bounds__(64) void k_mvs_enter(Bucket B)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B.count)
        return;
    double m[N], x[N][3], v[N][3], a[N][3];
    load_rows<N>(B, s, m, x, v, a, false);
    to_mvs<N>(m, x, v);
    mvs_acc<N>(m, x, a);
    a[0][0] = a[0][1] = a[0][2] = 0.0;
    store_rows<N>(B, s, x, v, a, true);
}

template <int N>
__global__ __launch_bounds__(64) void k_mvs_leave(Bucket B)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B.count)
        return;
    double m[N], x[N][3], v[N][3], a[N][3];
    load_rows<N>(B, s, m, x, v, a, false);
    from_mvs<N>(m, x, v);
    store_rows<N>(B, s, x, v, a, false);
}

// Fixed-step MVS integration of one system per lane for at most P.quantum
// steps: the run's whole steps, then the shortened final step if one is due
// (the clock logic of the Hermite kernels).
template <int N>
__global__ __launch_bounds__(256) void k_plain_mvs(Bucket B, StepParams P)
{
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= B.count)
        return;
    Clock c = load_clock(B, slot);
    if (c.status != ST_ACTIVE)
        return;
    double m[N], Q[N][3], V[N][3], acc[N][3];
    load_rows<N>(B, slot, m, Q, V, acc, true);
    const double inv_m0 = 1.0 / m[0];
    int budget = P.quantum;
#pragma unroll 1
    for (int seg = 0; seg < 2 && c.status == ST_ACTIVE && budget > 0; ++seg) {
        long long cnt = 0;
        double h = c.dt;
        if (seg == 0) {
            cnt = c.nfull - c.k;
            cnt = cnt < 0 ? 0 : cnt;
        } else {
            const double rem = c.t_end - c.t;
            if (rem * c.dt > 1e-9 * c.dt * c.dt) {
                cnt = 1;
                h = rem;
            } else {
                c.t = c.t_end;
                c.status = ST_DONE;
            }
        }
        cnt = min(cnt, (long long)budget);
        cnt = min(cnt, P.max_steps - c.steps);
        const int nrun = cnt > 0 ? (int)cnt : 0;
        int done = 0;
#pragma unroll 1
        for (; done < nrun; ++done) {
            const int st = mvs_step<N>(m, Q, V, acc, inv_m0, h);
            if (st != ST_ACTIVE) {
                c.status = st;
                break;
            }
        }
        budget -= done;
        c.steps += done;
        if (seg == 0) {
            c.k += done;
            if (done > 0)
                c.t = fma((double)c.k, c.dt, c.t0);
            if (c.status == ST_ACTIVE && c.k >= c.nfull) {
                const double rem = c.t_end - c.t;
                if (!(rem * c.dt > 1e-9 * c.dt * c.dt)) {
                    c.t = c.t_end;
                    c.status = ST_DONE;
                }
            }
        } else if (done > 0 && c.status == ST_ACTIVE) {
            c.t = c.t_end;
            c.status = ST_DONE;
        }
        if (c.status == ST_ACTIVE && c.steps >= P.max_steps)
            c.status = ST_MAXSTEPS;
    }
    bool fin = true;
#pragma unroll
    for (int b = 0; b < N; ++b)
        fin = fin && finite3(Q[b]) && finite3(V[b]);
    if (!fin)
        c.status = ST_NONFINITE;
    store_rows<N>(B, slot, Q, V, acc, true);
    store_clock(B, slot, c);
}

// State read-back of a bucket in MVS form: converted to inertial (x, v) on
// the way out; the stored form is left as it is.
template <int N>
__global__ __launch_bounds__(64) void k_unpack_mvs(Bucket B, const long long *__restrict__ orig_off,
                                                   double *pos, double *vel, double *t, int *status,
                                                   long long *steps)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B.count)
        return;
    double m[N], x[N][3], v[N][3], a[N][3];
    load_rows<N>(B, s, m, x, v, a, false);
    from_mvs<N>(m, x, v);
    const int o = B.orig[s];
    const long long base = orig_off[o];
#pragma unroll
    for (int b = 0; b < N; ++b)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            if (pos)
                pos[3 * (base + b) + c] = x[b][c];
            if (vel)
                vel[3 * (base + b) + c] = v[b][c];
        }
    if (t)
        t[o] = B.t[s];
    if (status)
        status[o] = B.status[s];
    if (steps)
        steps[o] = B.steps[s];
}

// ---------------------------------------------------------------------------
// Runge-Kutta Cash-Karp 4(5), Sections 2.2.2 and 4.3.2 (body per lane)
// ---------------------------------------------------------------------------
// The embedded pair of Cash & Karp (ACM TOMS 16, 1990) on y = (x, v),
// y' = (v, a(x)): six stages, each one acceleration evaluation (Eq. 1; a
// lane holds one body and reads its partners' positions from the
// wavefront's LDS slice, planets in ascending order, the star last).  The
// step advances with the fifth-order weights; the error estimate is the
// difference from the fourth-order weights.  Adaptive control: with X and V
// the largest |x_i| and |v_i| of the system at the step's start,
// E = max_i max(|dx_i| / (eps X), |dv_i| / (eps V)); E <= 1 accepts and
// proposes h min(5, max(0.2, 0.9 E^(-1/5))) (a step shortened onto t_end
// leaves the proposal as it was); E > 1 rejects (state and time unchanged)
// and retries with h max(0.1, 0.9 E^(-1/4)).
struct RkTableau {
    // coupling coefficients a[stage][j], j < stage
    static constexpr double a[6][5] = {
        {0, 0, 0, 0, 0},
        {1.0 / 5.0, 0, 0, 0, 0},
        {3.0 / 40.0, 9.0 / 40.0, 0, 0, 0},
        {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0, 0},
        {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0},
        {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0}};
    // fifth-order weights, and fifth- minus fourth-order weights
    static constexpr double b[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0,
                                    512.0 / 1771.0};
    static constexpr double e[6] = {37.0 / 378.0 - 2825.0 / 27648.0, 0.0,
                                    250.0 / 621.0 - 18575.0 / 48384.0,
                                    125.0 / 594.0 - 13525.0 / 55296.0, -277.0 / 14336.0,
                                    512.0 / 1771.0 - 1.0 / 4.0};
};

// Acceleration of this lane's body (Eq. 1) from its partners' positions.
template <int N>
__device__ __forceinline__ void rk_accel(BplLds &L, const int lane, const int b, const int s,
                                         const double (&xi)[3], double (&acc)[3])
{
    constexpr int S = 64 / N;
    L.xy[lane] = make_double2(xi[0], xi[1]);
    L.zvx[lane] = make_double2(xi[2], 0.0);
    wave_sync();
    acc[0] = acc[1] = acc[2] = 0.0;
    const int skip = b == 0 ? (1 << 20) : b;
#pragma unroll FB_BPL_UNROLL
    for (int k = 0; k <= N - 2; ++k) {
        // k < N-2: the other planets in ascending order; k = N-2: the star
        // (for the star lane: the last planet)
        const int j = k < N - 2 ? k + 1 + (k + 1 >= skip ? 1 : 0) : (b == 0 ? N - 1 : 0);
        const int idx = j * S + s;
        const double2 p0 = L.xy[idx];
        const double2 p1 = L.zvx[idx];
        const double rx = p0.x - xi[0], ry = p0.y - xi[1], rz = p1.x - xi[2];
        const double ri = rsqrt_nr(fma(rz, rz, fma(ry, ry, rx * rx)));
        const double mr3 = L.mr[idx].x * (ri * ri * ri);
        acc[0] = fma(mr3, rx, acc[0]);
        acc[1] = fma(mr3, ry, acc[1]);
        acc[2] = fma(mr3, rz, acc[2]);
    }
    wave_sync();
}

__device__ __forceinline__ double norm3d(const double (&p)[3])
{
    return sqrt(fma(p[2], p[2], fma(p[1], p[1], p[0] * p[0])));
}

// Six stages of (x, v) derivatives per lane do not fit the 4-waves budget
// of the Hermite body-per-lane kernels without spilling; two waves per SIMD
// give them registers.
#ifndef FB_RK_WAVES
#define FB_RK_WAVES 2
#endif

template <int N, bool ADV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(FB_RK_WAVES)))
void k_plain_rkck(Bucket B, StepParams P, double eps)
{
    constexpr int S = 64 / N;
    using T = RkTableau;
    const int wave = threadIdx.x >> 6;
    const int tile = blockIdx.x * (blockDim.x >> 6) + wave;
    const int first = tile * S;
    if (first >= B.count)
        return;
    const int count = min(S, B.count - first);
    BplLds &L = *reinterpret_cast<BplLds *>(wave_lds_base<sizeof(BplLds), false>());
    const int lane = threadIdx.x & 63;
    const int braw = lane / S;
    const int b = braw < N ? braw : N - 1;
    const int s = lane - braw * S;
    const bool valid = braw < N && s < count;
    const int slot = first + s;
    const size_t pitch = B.pitch;
    double mi = 0.0, x[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0};
    Clock c;
    c.status = ST_DONE;
    if (valid) {
        mi = B.st[(R_M * N + b) * pitch + slot];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            x[cc] = B.st[((R_X + cc) * N + b) * pitch + slot];
            v[cc] = B.st[((R_V + cc) * N + b) * pitch + slot];
        }
        c = load_clock(B, slot);
    }
    L.mr[lane].x = mi;
    wave_sync();
    for (int q = 0; q < P.quantum; ++q) {
        double h = 0.0;
        bool last = false;
        const bool act = valid && plan_step(c, P, h, last);
        if (!__any(act))
            break;
        if (!act)
            h = 0.0;
        double kx[6][3], kv[6][3];
#pragma unroll
        for (int st = 0; st < 6; ++st) {
            double xs[3];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                double dx = 0.0, dv = 0.0;
#pragma unroll
                for (int j = 0; j < st; ++j) {
                    dx = fma(T::a[st][j], kx[j][cc], dx);
                    dv = fma(T::a[st][j], kv[j][cc], dv);
                }
                xs[cc] = fma(h, dx, x[cc]);
                kx[st][cc] = fma(h, dv, v[cc]);
            }
            rk_accel<N>(L, lane, b, s, xs, kv[st]);
        }
        double x5[3], v5[3], ex[3], ev[3];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            double sx = 0.0, sv = 0.0, ux = 0.0, uv = 0.0;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                sx = fma(T::b[j], kx[j][cc], sx);
                sv = fma(T::b[j], kv[j][cc], sv);
                ux = fma(T::e[j], kx[j][cc], ux);
                uv = fma(T::e[j], kv[j][cc], uv);
            }
            x5[cc] = fma(h, sx, x[cc]);
            v5[cc] = fma(h, sv, v[cc]);
            ex[cc] = h * ux;
            ev[cc] = h * uv;
        }
        bool accept = true;
        double dtp = 0.0;
        if (ADV) {
            const double X = sys_max<N>(L, lane, s, norm3d(x));
            const double V = sys_max<N>(L, lane, s, norm3d(v));
            const double E = sys_max<N>(L, lane, s,
                                        fmax(norm3d(ex) / (eps * X), norm3d(ev) / (eps * V)));
            accept = E <= 1.0;
            if (act && !accept) {
                if (!__builtin_isfinite(E))
                    c.status = ST_NONFINITE;
                else
                    c.dtn = h * fmax(0.1, 0.9 * pow(E, -0.25));
            }
            dtp = last ? c.dtn : h * (E > 0.0 ? fmin(5.0, fmax(0.2, 0.9 * pow(E, -0.2))) : 5.0);
        }
        if (act && accept) {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                x[cc] = x5[cc];
                v[cc] = v5[cc];
            }
            finish_step(c, P, last, h, dtp);
        }
    }
    if (!ADV) {
        const int fl = sys_or_flags<N>(s, (finite3(x) && finite3(v)) ? 0 : 1);
        if (valid && fl)
            c.status = ST_NONFINITE;
    }
    if (valid) {
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            B.st[((R_X + cc) * N + b) * pitch + slot] = x[cc];
            B.st[((R_V + cc) * N + b) * pitch + slot] = v[cc];
        }
        if (b == 0)
            store_clock(B, slot, c);
    }
}

// ---------------------------------------------------------------------------
// large systems (n > 16): one body per lane across a whole workgroup
// ---------------------------------------------------------------------------
// Section 4.2's second gravitation variant, for larger n.  Every lane owns
// one body and sums all n-1 of that body's interactions itself, so each pair
// is evaluated twice (once from either side) and the workgroup's LDS holds
// only the bodies' evaluation state, never per-pair terms.  S = floor(T / n)
// systems share a workgroup of T lanes (lane = system * n + body); a body's
// partners are LDS broadcasts to the lanes of its system.  Two copies of the
// evaluation state alternate, so an evaluation costs one workgroup barrier: a
// lane overwrites a copy only after the next evaluation's barrier, which
// every reader of that copy has passed.

// Lanes of the largest large-n workgroup (its LDS stays below 64 KiB).
constexpr int kLargeMaxLanes = 512;

// Dynamic LDS of a large-n workgroup holding T bodies: two copies of the
// evaluation state (three 16-byte pairs per body each), the masses, one
// reduction double and one int per body.
__host__ __device__ constexpr size_t large_lds_bytes(int T)
{
    return (size_t)T * (6 * sizeof(double2) + 2 * sizeof(double) + sizeof(int));
}

struct LargeView {
    double2 *xy, *zvx, *vyvz;   // copy c of lane l at [c * T + l]
    double *m;
    double *red;
    int *flag;
};

__device__ __forceinline__ LargeView large_view(const int T)
{
    extern __shared__ char fb_dyn_lds[];
    double2 *p = reinterpret_cast<double2 *>(fb_dyn_lds);
    LargeView V;
    V.xy = p;
    V.zvx = p + 2 * T;
    V.vyvz = p + 4 * T;
    V.m = reinterpret_cast<double *>(p + 6 * T);
    V.red = V.m + T;
    V.flag = reinterpret_cast<int *>(V.red + T);
    return V;
}

// One interaction of body i with the partner at LDS index idx of one copy
// (Eq. 1 and its time derivative; the terms of bpl_interact).
__device__ __forceinline__ void large_interact(const double2 *__restrict__ xy,
                                               const double2 *__restrict__ zvx,
                                               const double2 *__restrict__ vyvz,
                                               const double *__restrict__ mm, const int idx,
                                               const double (&xi)[3], const double (&vi)[3],
                                               double (&a)[3], double (&jk)[3])
{
    const double2 p0 = xy[idx];
    const double2 p1 = zvx[idx];
    const double2 p2 = vyvz[idx];
    const double mj = mm[idx];
    const double rx = p0.x - xi[0], ry = p0.y - xi[1], rz = p1.x - xi[2];
    const double ux = p1.y - vi[0], uy = p2.x - vi[1], uz = p2.y - vi[2];
    const double r2 = fma(rz, rz, fma(ry, ry, rx * rx));
    const double ru = fma(rz, uz, fma(ry, uy, rx * ux));
    const double ri = rsqrt_nr(r2);
    const double ri2 = ri * ri;
    const double mr3 = mj * (ri2 * ri);
    const double al = 3.0 * ru * ri2;
    a[0] = fma(mr3, rx, a[0]);
    a[1] = fma(mr3, ry, a[1]);
    a[2] = fma(mr3, rz, a[2]);
    jk[0] = fma(mr3, fma(-al, rx, ux), jk[0]);
    jk[1] = fma(mr3, fma(-al, ry, uy), jk[1]);
    jk[2] = fma(mr3, fma(-al, rz, uz), jk[2]);
}

// Publish this lane's state in copy `cp`, wait for the workgroup, and (live
// lanes) sum the body's interactions: the other planets in ascending order,
// then the star (the star's lane sums planets 1..n-1).
__device__ __forceinline__ void large_eval(const LargeView &V, const int T, const int cp,
                                           const int tid, const int base, const int b,
                                           const int n, const bool live, const double (&xi)[3],
                                           const double (&vi)[3], double (&a)[3],
                                           double (&jk)[3])
{
    const double2 *xy = V.xy + cp * T;
    const double2 *zvx = V.zvx + cp * T;
    const double2 *vyvz = V.vyvz + cp * T;
    V.xy[cp * T + tid] = make_double2(xi[0], xi[1]);
    V.zvx[cp * T + tid] = make_double2(xi[2], vi[0]);
    V.vyvz[cp * T + tid] = make_double2(vi[1], vi[2]);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        a[c] = 0.0;
        jk[c] = 0.0;
    }
    if (!live)
        return;
    const int skip = b == 0 ? INT_MAX : b;
#pragma unroll 4
    for (int k = 0; k < n - 2; ++k) {
        const int j = k + 1 + (k + 1 >= skip ? 1 : 0);
        large_interact(xy, zvx, vyvz, V.m, base + j, xi, vi, a, jk);
    }
    large_interact(xy, zvx, vyvz, V.m, base + (b == 0 ? n - 1 : 0), xi, vi, a, jk);
}

// Lane geometry of a large-n workgroup.
struct LargeLane {
    int tid, sys, b, base, slot;
    bool valid;
};

__device__ __forceinline__ LargeLane large_lane(const Bucket &B, const int S)
{
    LargeLane l;
    l.tid = threadIdx.x;
    l.sys = l.tid / B.n;
    l.b = l.tid - l.sys * B.n;
    l.base = l.sys * B.n;
    const int slot = blockIdx.x * S + l.sys;
    l.valid = l.sys < S && slot < B.count;
    l.slot = l.valid ? slot : 0;
    return l;
}

// Evaluation state of one body in the step kernel's LDS (48 bytes, so a
// partner is three ds_read_b128 at immediate offsets from one address).
struct LargeBody {
    double2 xy, zvx, vyvz;
};

// The step kernel's view of its dynamic LDS (E bodies): two copies of the
// bodies' evaluation state, the masses and one int per body; the same bytes
// as large_lds_bytes(E).
struct LargeStepView {
    LargeBody *st;   // copy c of body entry e at [c * E + e]
    double *m;
    double *red;
    int *flag;
};

__device__ __forceinline__ LargeStepView large_step_view(const int E)
{
    extern __shared__ char fb_dyn_lds[];
    LargeStepView V;
    V.st = reinterpret_cast<LargeBody *>(fb_dyn_lds);
    V.m = reinterpret_cast<double *>(V.st + 2 * E);
    V.red = V.m + E;
    V.flag = reinterpret_cast<int *>(V.red + E);
    return V;
}
static_assert(2 * sizeof(LargeBody) + 2 * sizeof(double) + sizeof(int) ==
                  6 * sizeof(double2) + 2 * sizeof(double) + sizeof(int),
              "step-kernel LDS view must match large_lds_bytes");

// Squared separations are floored here before the inverse distance is taken:
// a body's interaction with itself (r = u = 0) then contributes exact zeros
// with every intermediate finite, and no real pair comes this close.
constexpr double kLargeMinR2 = 1e-100;

// One interaction of body i with a partner (Eq. 1 and its time derivative,
// the terms of bpl_interact).  With TS, also the pair's step-rule quantity
// (|u|^2 + 3 (r.u)^2/|r|^2) / |r|^2 into wmax (zero for the self term).
template <bool TS>
__device__ __forceinline__ void large_interact_p(const LargeBody &p, const double mj,
                                                 const double (&xi)[3], const double (&vi)[3],
                                                 double (&a)[3], double (&jk)[3], double &wmax)
{
    const double rx = p.xy.x - xi[0], ry = p.xy.y - xi[1], rz = p.zvx.x - xi[2];
    const double ux = p.zvx.y - vi[0], uy = p.vyvz.x - vi[1], uz = p.vyvz.y - vi[2];
    const double r2 = fmax(fma(rz, rz, fma(ry, ry, rx * rx)), kLargeMinR2);
    const double ru = fma(rz, uz, fma(ry, uy, rx * ux));
    const double ri = rsqrt_nr(r2);
    const double ri2 = ri * ri;
    const double mr3 = mj * (ri2 * ri);
    const double al = 3.0 * ru * ri2;
    a[0] = fma(mr3, rx, a[0]);
    a[1] = fma(mr3, ry, a[1]);
    a[2] = fma(mr3, rz, a[2]);
    jk[0] = fma(mr3, fma(-al, rx, ux), jk[0]);
    jk[1] = fma(mr3, fma(-al, ry, uy), jk[1]);
    jk[2] = fma(mr3, fma(-al, rz, uz), jk[2]);
    if (TS) {
        const double u2 = fma(uz, uz, fma(uy, uy, ux * ux));
        wmax = fmax(wmax, fma(al, ru, u2) * ri2);
    }
}

// Waves per SIMD the register allocator targets for the large-n step kernel.
#ifndef FB_LARGE_WAVES
#define FB_LARGE_WAVES 2
#endif

// The evaluation of the K-body step kernel: publish this lane's bodies in
// copy `cp` (entry system base + body), wait for the workgroup, then sum
// each owned body's interactions: planets 1..n-1 in ascending order (its own
// index contributing zeros), then the star.
template <int K, bool TS>
__device__ __forceinline__ void large_eval_k(const LargeStepView &V, const int E, const int cp,
                                             const int base, const int n, const bool live,
                                             const int (&bk)[K], const bool (&own)[K],
                                             const double (&xi)[K][3], const double (&vi)[K][3],
                                             double (&a)[K][3], double (&jk)[K][3],
                                             double (&w)[K])
{
    LargeBody *st = V.st + cp * E + base;
    const double *mm = V.m + base;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (own[k]) {
            LargeBody &q = st[bk[k]];
            q.xy = make_double2(xi[k][0], xi[k][1]);
            q.zvx = make_double2(xi[k][2], vi[k][0]);
            q.vyvz = make_double2(vi[k][1], vi[k][2]);
        }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
        w[k] = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            a[k][c] = 0.0;
            jk[k][c] = 0.0;
        }
    }
    if (!live)
        return;
#pragma unroll 2
    for (int j = 1; j < n; ++j) {
        const LargeBody p = st[j];
        const double mj = mm[j];
#pragma unroll
        for (int k = 0; k < K; ++k)
            large_interact_p<TS>(p, mj, xi[k], vi[k], a[k], jk[k], w[k]);
    }
    const LargeBody p = st[0];
    const double m0 = mm[0];
#pragma unroll
    for (int k = 0; k < K; ++k)
        large_interact_p<TS>(p, m0, xi[k], vi[k], a[k], jk[k], w[k]);
}

// Per-system reduction of one value per owned body, in body order (max, or
// sum); every valid lane gets its system's result.  Two barriers.
template <int K, bool MAXOP>
__device__ __forceinline__ double large_sys_reduce(double *red, const int base, const int n,
                                                   const bool valid, const int (&bk)[K],
                                                   const bool (&own)[K], const double (&val)[K])
{
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (own[k])
            red[base + bk[k]] = val[k];
    __syncthreads();
    double r = 0.0;
    if (valid) {
        r = red[base];
        for (int b = 1; b < n; ++b)
            r = MAXOP ? fmax(r, red[base + b]) : r + red[base + b];
    }
    __syncthreads();
    return r;
}

// Stop-rule flags of each system after a committed step (the bits of
// bpl_stop_flags: 1 non-finite, 2 two planets within one mutual Hill radius,
// 4 a planet beyond r_eject), OR-ed over the system; positions go through
// copy 0 of the evaluation state, free until the next step's first
// evaluation.
template <int K>
__device__ __forceinline__ int large_stop_flags(const LargeStepView &V, const int base,
                                                const int n, const bool valid, const int (&bk)[K],
                                                const bool (&own)[K], const double (&x)[K][3],
                                                const double (&v)[K][3], const StepParams &P)
{
    int fl = 0;
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (own[k]) {
            fl |= (finite3(x[k]) && finite3(v[k])) ? 0 : 1;
            V.st[base + bk[k]].xy = make_double2(x[k][0], x[k][1]);
            V.st[base + bk[k]].zvx.x = x[k][2];
        }
    __syncthreads();
    double rb[K];
    if (valid) {
        const LargeBody s0 = V.st[base];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const double dx = x[k][0] - s0.xy.x, dy = x[k][1] - s0.xy.y, dz = x[k][2] - s0.zvx.x;
            rb[k] = sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
            if (own[k])
                V.red[base + bk[k]] = rb[k];
        }
    }
    __syncthreads();
    if (valid) {
        const double inv24m0 = 1.0 / (24.0 * V.m[base]);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!own[k] || bk[k] == 0)
                continue;
            if ((P.stop_rules & 2) && rb[k] > P.r_eject)
                fl |= 4;
            if (P.stop_rules & 1) {
                const double mi = V.m[base + bk[k]];
                for (int j = 1; j < n; ++j) {
                    if (j == bk[k])
                        continue;
                    const LargeBody q = V.st[base + j];
                    const double ex = x[k][0] - q.xy.x, ey = x[k][1] - q.xy.y, ez = x[k][2] - q.zvx.x;
                    const double sep2 = fma(ez, ez, fma(ey, ey, ex * ex));
                    if (hill_close(sep2, mi, V.m[base + j], inv24m0, rb[k], V.red[base + j]))
                        fl |= 2;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (own[k])
                V.flag[base + bk[k]] = k == 0 ? fl : 0;
    }
    __syncthreads();
    int r = 0;
    if (valid)
        for (int b = 0; b < n; ++b)
            r |= V.flag[base + b];
    __syncthreads();
    return r;
}

// Fixed Hermite P(EC)^2 steps (Algorithm 1's loop, Algorithm 2's step) for
// at most P.quantum steps.  Lane h of a system owns bodies h, h + H, ...,
// h + (K-1) H with H = ceil(n / K); S = floor(T / H) systems per workgroup
// of T lanes.  The LDS arrays hold K T bodies, system s's at s n + body.
// Every lane commits every iteration (so the pre-step state need not stay
// live through the evaluations); a system's state is written back as soon
// as it stops stepping, and its registers are ignored after that.
template <int K, bool ADV>
__global__ __launch_bounds__(kLargeMaxLanes / K) __attribute__((amdgpu_waves_per_eu(FB_LARGE_WAVES)))
void k_plain_large(Bucket B, StepParams P, int S)
{
    const int T = blockDim.x, n = B.n, H = (n + K - 1) / K, E = K * T;
    const LargeStepView V = large_step_view(E);
    const int tid = threadIdx.x;
    const int sys = tid / H, h = tid - sys * H;
    const int slot0 = blockIdx.x * S + sys;
    const bool valid = sys < S && slot0 < B.count;
    const int slot = valid ? slot0 : 0;
    const int base = sys * n;
    const size_t pitch = B.pitch;
    int bk[K];
    bool own[K];
    double x[K][3], v[K][3], a0[K][3], j0[K][3];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        bk[k] = h + k * H;
        own[k] = valid && bk[k] < n;
        const int b = own[k] ? bk[k] : 0;
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            x[k][cc] = v[k][cc] = a0[k][cc] = j0[k][cc] = 0.0;
            if (own[k]) {
                x[k][cc] = B.st[((R_X + cc) * n + b) * pitch + slot];
                v[k][cc] = B.st[((R_V + cc) * n + b) * pitch + slot];
                a0[k][cc] = B.st[((R_A + cc) * n + b) * pitch + slot];
                j0[k][cc] = B.st[((R_J + cc) * n + b) * pitch + slot];
            }
        }
        if (own[k])   // ordered before any read by the loop's first barrier
            V.m[base + b] = B.st[(R_M * n + b) * pitch + slot];
    }
    Clock c;
    c.status = ST_DONE;
    if (valid)
        c = load_clock(B, slot);
    bool pending = false;   // registers hold committed steps not yet written back
    int bad = 0;            // non-finite state written back
    auto write_back = [&]() {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (!own[k])
                continue;
            const int b = bk[k];
            bad |= (finite3(x[k]) && finite3(v[k])) ? 0 : 1;
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                B.st[((R_X + cc) * n + b) * pitch + slot] = x[k][cc];
                B.st[((R_V + cc) * n + b) * pitch + slot] = v[k][cc];
                B.st[((R_A + cc) * n + b) * pitch + slot] = a0[k][cc];
                B.st[((R_J + cc) * n + b) * pitch + slot] = j0[k][cc];
            }
        }
        pending = false;
    };
    for (int q = 0; q < P.quantum; ++q) {
        double hs = 0.0;
        bool last = false;
        const bool act = valid && plan_step(c, P, hs, last);
        if (pending && !act)
            write_back();
        if (!__syncthreads_or(act))
            break;
        const Coef cf = make_coef(hs);
        double xc[K][3], vc[K][3], bx[K][3], bv[K][3], ak[K][3], jk[K][3];
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                predict_comp(cf, x[k][cc], v[k][cc], a0[k][cc], j0[k][cc], xc[k][cc], vc[k][cc],
                             bx[k][cc], bv[k][cc]);
        double w[K];
        large_eval_k<K, false>(V, E, 0, base, n, act, bk, own, xc, vc, ak, jk, w);
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc)
                correct_comp(cf, bx[k][cc], bv[k][cc], ak[k][cc], jk[k][cc], xc[k][cc], vc[k][cc]);
        large_eval_k<K, ADV>(V, E, 1, base, n, act, bk, own, xc, vc, ak, jk, w);
#pragma unroll
        for (int k = 0; k < K; ++k)
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                correct_comp(cf, bx[k][cc], bv[k][cc], ak[k][cc], jk[k][cc], x[k][cc], v[k][cc]);
                a0[k][cc] = ak[k][cc];
                j0[k][cc] = jk[k][cc];
            }
        double dtp = 0.0;
        if (ADV && P.adaptive == 1)   // the pairwise rule: max over the system's pairs
            dtp = P.eta * rsqrt_nr(large_sys_reduce<K, true>(V.red, base, n, valid, bk, own, w));
        if (ADV && P.adaptive == 2) { // Eq. 5: sum over the system's bodies
            double q[K];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const double aa = fma(ak[k][2], ak[k][2], fma(ak[k][1], ak[k][1], ak[k][0] * ak[k][0]));
                const double jj = fma(jk[k][2], jk[k][2], fma(jk[k][1], jk[k][1], jk[k][0] * jk[k][0]));
                q[k] = jj / aa;
            }
            dtp = P.eta * rsqrt_nr(large_sys_reduce<K, false>(V.red, base, n, valid, bk, own, q));
        }
        if (act) {
            finish_step(c, P, last, hs, dtp);
            pending = true;
        }
        if (ADV) {
            const int fl = large_stop_flags<K>(V, base, n, valid, bk, own, x, v, P);
            if (act && fl)
                c.status = status_of_flags(fl);
        }
    }
    if (pending)
        write_back();
#pragma unroll
    for (int k = 0; k < K; ++k)
        if (own[k])
            V.flag[base + bk[k]] = bad;
    __syncthreads();
    if (valid && h == 0) {   // the lane of the star
        int fl = 0;
        if (!ADV)            // (with ADV the stop flags checked every step)
            for (int b = 0; b < n; ++b)
                fl |= V.flag[base + b];
        if (fl)
            c.status = ST_NONFINITE;
        store_clock(B, slot, c);
    }
}

// Algorithm 1's "prepare" for large n: (a0, j0) at the current state.
__global__ __launch_bounds__(kLargeMaxLanes) void k_prepare_large(Bucket B, int S)
{
    const int T = blockDim.x, n = B.n;
    const LargeView V = large_view(T);
    const LargeLane l = large_lane(B, S);
    const size_t pitch = B.pitch;
    double mi = 0.0, x[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0};
    if (l.valid) {
        mi = B.st[(R_M * n + l.b) * pitch + l.slot];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            x[cc] = B.st[((R_X + cc) * n + l.b) * pitch + l.slot];
            v[cc] = B.st[((R_V + cc) * n + l.b) * pitch + l.slot];
        }
    }
    V.m[l.tid] = mi;
    double a[3], jk[3];
    large_eval(V, T, 0, l.tid, l.base, l.b, n, l.valid, x, v, a, jk);
    if (!l.valid)
        return;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        B.st[((R_A + cc) * n + l.b) * pitch + l.slot] = a[cc];
        B.st[((R_J + cc) * n + l.b) * pitch + l.slot] = jk[cc];
    }
}

// Per-system sums over the bodies of a large-n workgroup, in body order, on
// the star's lane: lane values q[0..4] go through copy 1 of the state arrays.
__device__ __forceinline__ void large_sum5(const LargeView &V, const int T, const LargeLane &l,
                                           const int n, const double (&q)[5], double (&out)[5])
{
    double2 *r0 = V.xy + T, *r1 = V.zvx + T, *r2 = V.vyvz + T;
    r0[l.tid] = make_double2(q[0], q[1]);
    r1[l.tid] = make_double2(q[2], q[3]);
    r2[l.tid] = make_double2(q[4], 0.0);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 5; ++c)
        out[c] = 0.0;
    if (!l.valid || l.b != 0)
        return;
    for (int k = 0; k < n; ++k) {
        const double2 p = r0[l.base + k], u = r1[l.base + k], w = r2[l.base + k];
        out[0] += p.x;
        out[1] += p.y;
        out[2] += u.x;
        out[3] += u.y;
        out[4] += w.x;
    }
}

// Energy (Eq. 6) and angular momentum parts of this lane's body: its kinetic
// energy, the potential of its pairs with higher-numbered partners (each pair
// once) and m x cross v.
__device__ __forceinline__ void large_energy_terms(const LargeView &V, const int T,
                                                   const LargeLane &l, const int n,
                                                   const double mi, const double (&x)[3],
                                                   const double (&v)[3], double (&q)[5])
{
    V.m[l.tid] = mi;
    V.xy[l.tid] = make_double2(x[0], x[1]);
    V.zvx[l.tid] = make_double2(x[2], 0.0);
    __syncthreads();
    double pot = 0.0;
    if (l.valid)
        for (int j = l.b + 1; j < n; ++j) {
            const double2 p0 = V.xy[l.base + j], p1 = V.zvx[l.base + j];
            const double dx = x[0] - p0.x, dy = x[1] - p0.y, dz = x[2] - p1.x;
            pot += V.m[l.base + j] / sqrt(fma(dz, dz, fma(dy, dy, dx * dx)));
        }
    q[0] = 0.5 * mi * fma(v[2], v[2], fma(v[1], v[1], v[0] * v[0])) - mi * pot;
    q[1] = 0.0;
    q[2] = mi * (x[1] * v[2] - x[2] * v[1]);
    q[3] = mi * (x[2] * v[0] - x[0] * v[2]);
    q[4] = mi * (x[0] * v[1] - x[1] * v[0]);
}

__device__ __forceinline__ void large_load_xv(const Bucket &B, const LargeLane &l, double &mi,
                                              double (&x)[3], double (&v)[3])
{
    mi = 0.0;
    const size_t pitch = B.pitch;
    const int n = B.n;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = 0.0;
        v[c] = 0.0;
    }
    if (!l.valid)
        return;
    mi = B.st[(R_M * n + l.b) * pitch + l.slot];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = B.st[((R_X + c) * n + l.b) * pitch + l.slot];
        v[c] = B.st[((R_V + c) * n + l.b) * pitch + l.slot];
    }
}

// Run start of a large-n bucket (one body per lane): the clock part on the
// star's lane, then, for systems that need one, the first adaptive step from
// the stored (a0, j0) (Eq. 5) or from the pairwise rule at the current state
// (the proposals of k_begin_run).
__global__ __launch_bounds__(kLargeMaxLanes) void k_begin_run_large(Bucket B, int S,
                                                                    int fixed_steps,
                                                                    long long n_steps,
                                                                    double t_end, double dt,
                                                                    int adaptive, double eta)
{
    const int T = blockDim.x, n = B.n;
    const LargeView V = large_view(T);
    const LargeLane l = large_lane(B, S);
    if (l.valid && l.b == 0)
        V.flag[l.base] = begin_run_clock(B, l.slot, fixed_steps, n_steps, t_end, dt, adaptive);
    __syncthreads();
    const bool need = l.valid && V.flag[l.base] != 0;
    if (!__syncthreads_or(need))
        return;
    const size_t pitch = B.pitch;
    double mi, x[3], v[3];
    large_load_xv(B, l, mi, x, v);
    double q = 0.0;
    if (adaptive == 2) {
        if (l.valid) {
            double a[3], jk[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                a[c] = B.st[((R_A + c) * n + l.b) * pitch + l.slot];
                jk[c] = B.st[((R_J + c) * n + l.b) * pitch + l.slot];
            }
            q = fma(jk[2], jk[2], fma(jk[1], jk[1], jk[0] * jk[0])) /
                fma(a[2], a[2], fma(a[1], a[1], a[0] * a[0]));
        }
    } else {
        V.m[l.tid] = mi;
        V.xy[l.tid] = make_double2(x[0], x[1]);
        V.zvx[l.tid] = make_double2(x[2], v[0]);
        V.vyvz[l.tid] = make_double2(v[1], v[2]);
        __syncthreads();
        if (l.valid) {
            for (int j = 0; j < n; ++j) {
                if (j == l.b)
                    continue;
                const double2 p0 = V.xy[l.base + j], p1 = V.zvx[l.base + j],
                              p2 = V.vyvz[l.base + j];
                const double rx = p0.x - x[0], ry = p0.y - x[1], rz = p1.x - x[2];
                const double ux = p1.y - v[0], uy = p2.x - v[1], uz = p2.y - v[2];
                const double r2 = fma(rz, rz, fma(ry, ry, rx * rx));
                const double ru = fma(rz, uz, fma(ry, uy, rx * ux));
                const double u2 = fma(uz, uz, fma(uy, uy, ux * ux));
                const double ri = rsqrt_nr(r2);
                const double ri2 = ri * ri;
                const double al = 3.0 * ru * ri2;
                q = fmax(q, fma(al, ru, u2) * ri2);
            }
        }
    }
    V.red[l.tid] = q;
    __syncthreads();
    if (need && l.b == 0) {
        double r = V.red[l.base];
        for (int b = 1; b < n; ++b)
            r = adaptive == 2 ? r + V.red[l.base + b] : fmax(r, V.red[l.base + b]);
        B.dtn[l.slot] = eta * rsqrt_nr(r);
    }
}

__device__ __forceinline__ void large_from_mvs(const LargeView &V, const int T, const LargeLane &l,
                                               const int n, const double mi, double (&x)[3],
                                               double (&v)[3]);

// Energy and angular momentum of every system of a large-n bucket, in
// inertial form or (MVS) in MVS form, converted first.
template <bool MVS>
__global__ __launch_bounds__(kLargeMaxLanes) void k_diag_large(Bucket B, int S, double *energy,
                                                     double *angmom)
{
    const int T = blockDim.x;
    const LargeView V = large_view(T);
    const LargeLane l = large_lane(B, S);
    double mi, x[3], v[3], q[5], sum[5];
    large_load_xv(B, l, mi, x, v);
    if (MVS) {
        V.m[l.tid] = mi;
        large_from_mvs(V, T, l, B.n, mi, x, v);
    }
    large_energy_terms(V, T, l, B.n, mi, x, v, q);
    large_sum5(V, T, l, B.n, q, sum);
    if (!l.valid || l.b != 0)
        return;
    const int o = B.orig[l.slot];
    if (energy)
        energy[o] = sum[0];
    if (angmom) {
        angmom[3 * o + 0] = sum[2];
        angmom[3 * o + 1] = sum[3];
        angmom[3 * o + 2] = sum[4];
    }
}

// Monitor record k of every system of a large-n bucket (layouts of k_log).
__global__ __launch_bounds__(kLargeMaxLanes) void k_log_large(Bucket B, int S,
                                                    const long long *__restrict__ orig_off,
                                                    int kind, double lx, double ly, double lz,
                                                    int k, int max_records, double *out)
{
    const int T = blockDim.x, n = B.n;
    const LargeView V = large_view(T);
    const LargeLane l = large_lane(B, S);
    double mi, x[3], v[3], q[5], sum[5];
    large_load_xv(B, l, mi, x, v);
    const int o = l.valid ? B.orig[l.slot] : 0;
    const double t = l.valid ? B.t[l.slot] : 0.0;
    if (kind == 0) {
        if (!l.valid)
            return;
        double *r = out + (size_t)max_records * ((size_t)o + 6 * (size_t)orig_off[o]) +
                    (size_t)k * (1 + 6 * n);
        if (l.b == 0)
            r[0] = t;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            r[1 + 3 * l.b + c] = x[c];
            r[1 + 3 * n + 3 * l.b + c] = v[c];
        }
        return;
    }
    if (kind == 1) {
        q[0] = mi;
        q[1] = mi * v[0];
        q[2] = mi * v[1];
        q[3] = mi * v[2];
        q[4] = 0.0;
    } else {
        large_energy_terms(V, T, l, n, mi, x, v, q);
    }
    large_sum5(V, T, l, n, q, sum);
    if (!l.valid || l.b != 0)
        return;
    if (kind == 1) {
        const double rv = fma(v[2] - sum[3] / sum[0], lz,
                              fma(v[1] - sum[2] / sum[0], ly, (v[0] - sum[1] / sum[0]) * lx));
        double *r = out + ((size_t)o * max_records + k) * 2;
        r[0] = t;
        r[1] = rv;
    } else {
        double *r = out + ((size_t)o * max_records + k) * 5;
        r[0] = t;
        r[1] = sum[0];
        r[2] = sum[2];
        r[3] = sum[3];
        r[4] = sum[4];
    }
}

// ---------------------------------------------------------------------------
// MVS for larger systems (9..512 bodies): one body per lane across a workgroup
// ---------------------------------------------------------------------------
// The sub-steps of Section 2.2.3 as in k_plain_mvs, laid out like the large-n
// Hermite kernels: each planet's lane drifts it along its own Kepler orbit,
// the planet-planet accelerations are one-sided partner loops over LDS
// broadcasts (planets in ascending order; the same values as the paired
// form), and the sums over a system (the drift's momentum, the centre of
// mass) are fma chains in body order on the star's lane, broadcast through
// LDS.  Every lane reaches every barrier: a system's outcome (unbound,
// Kepler failure) predicates its updates, never the control flow.

// Over bodies b >= b0 of the lane's system: sum of w_b u_b (an fma chain in
// body order) and the star's own u, to every valid lane.  Three barriers.
__device__ __forceinline__ void large_sys_wsum3(const LargeView &V, const int T,
                                                const LargeLane &l, const int n, const int b0,
                                                const double w, const double (&u)[3],
                                                double (&sum)[3], double (&star_u)[3])
{
    double2 *in0 = V.xy + T, *in1 = V.zvx + T, *res = V.vyvz + T;
    in0[l.tid] = make_double2(u[0], u[1]);
    in1[l.tid] = make_double2(u[2], w);
    __syncthreads();
    if (l.valid && l.b == 0) {
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int b = b0; b < n; ++b) {
            const double2 p = in0[l.base + b], q = in1[l.base + b];
            s0 = fma(q.y, p.x, s0);
            s1 = fma(q.y, p.y, s1);
            s2 = fma(q.y, q.x, s2);
        }
        res[l.base] = make_double2(s0, s1);
        V.red[l.base] = s2;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c)
        sum[c] = star_u[c] = 0.0;
    if (l.valid) {
        const double2 r = res[l.base], p = in0[l.base], q = in1[l.base];
        sum[0] = r.x;
        sum[1] = r.y;
        sum[2] = V.red[l.base];
        star_u[0] = p.x;
        star_u[1] = p.y;
        star_u[2] = q.x;
    }
    __syncthreads();
}

// OR of a per-lane flag over the lane's system, to every valid lane.
__device__ __forceinline__ int large_sys_or(const LargeView &V, const LargeLane &l, const int n,
                                            const int f)
{
    V.flag[l.tid] = f;
    __syncthreads();
    int r = 0;
    if (l.valid)
        for (int b = 0; b < n; ++b)
            r |= V.flag[l.base + b];
    __syncthreads();
    return r;
}

// Planet-planet acceleration of this lane's planet at heliocentric positions
// Q (each lane's own, published here); zero on the star's lane.
__device__ __forceinline__ void large_mvs_acc(const LargeView &V, const LargeLane &l, const int n,
                                              const double (&Q)[3], double (&acc)[3])
{
    V.xy[l.tid] = make_double2(Q[0], Q[1]);
    V.zvx[l.tid] = make_double2(Q[2], 0.0);
    __syncthreads();
    acc[0] = acc[1] = acc[2] = 0.0;
    if (l.valid && l.b > 0)
        for (int j = 1; j < n; ++j) {
            if (j == l.b)
                continue;
            const double2 p0 = V.xy[l.base + j], p1 = V.zvx[l.base + j];
            const double d0 = p0.x - Q[0], d1 = p0.y - Q[1], d2 = p1.x - Q[2];
            const double sr = rsqrt_nr(fma(d2, d2, fma(d1, d1, d0 * d0)));
            const double mj = V.m[l.base + j] * (sr * sr * sr);
            acc[0] = fma(mj, d0, acc[0]);
            acc[1] = fma(mj, d1, acc[1]);
            acc[2] = fma(mj, d2, acc[2]);
        }
    __syncthreads();
}

// MVS form -> inertial (x, v) of this lane's body (from_mvs): x_0 = X -
// sum m_i Q_i / M, x_i = Q_i + x_0, v_0 = Vc - sum m_i V_i / m_0,
// v_i = V_i + Vc.  V.m must hold the masses.
__device__ __forceinline__ void large_from_mvs(const LargeView &V, const int T, const LargeLane &l,
                                               const int n, const double mi, double (&x)[3],
                                               double (&v)[3])
{
    const double one[3] = {mi, 0.0, 0.0};
    double Ms[3], st[3], sq[3], X[3], sp[3], Vc[3];
    large_sys_wsum3(V, T, l, n, 0, 1.0, one, Ms, st);
    large_sys_wsum3(V, T, l, n, 1, mi, x, sq, X);
    large_sys_wsum3(V, T, l, n, 1, mi, v, sp, Vc);
    const double M = Ms[0], m0 = l.valid ? V.m[l.base] : 1.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double x0 = X[c] - sq[c] / M;
        if (l.b == 0) {
            x[c] = x0;
            v[c] = Vc[c] - sp[c] / m0;
        } else {
            x[c] += x0;
            v[c] += Vc[c];
        }
    }
}

__device__ __forceinline__ void large_load_rows(const Bucket &B, const LargeLane &l, double &mi,
                                                double (&x)[3], double (&v)[3], double (&a)[3])
{
    mi = 0.0;
    const size_t pitch = B.pitch;
    const int n = B.n;
#pragma unroll
    for (int c = 0; c < 3; ++c)
        x[c] = v[c] = a[c] = 0.0;
    if (!l.valid)
        return;
    mi = B.st[(R_M * n + l.b) * pitch + l.slot];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        x[c] = B.st[((R_X + c) * n + l.b) * pitch + l.slot];
        v[c] = B.st[((R_V + c) * n + l.b) * pitch + l.slot];
        a[c] = B.st[((R_A + c) * n + l.b) * pitch + l.slot];
    }
}

__device__ __forceinline__ void large_store_rows(const Bucket &B, const LargeLane &l,
                                                 const double (&x)[3], const double (&v)[3],
                                                 const double (&a)[3], bool with_a)
{
    if (!l.valid)
        return;
    const size_t pitch = B.pitch;
    const int n = B.n;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        B.st[((R_X + c) * n + l.b) * pitch + l.slot] = x[c];
        B.st[((R_V + c) * n + l.b) * pitch + l.slot] = v[c];
        if (with_a)
            B.st[((R_A + c) * n + l.b) * pitch + l.slot] = a[c];
    }
}

// Inertial -> MVS form of a bucket (to_mvs), with the planet-planet
// accelerations at Q in the a0 rows.
__global__ __launch_bounds__(kLargeMaxLanes) void k_mvs_enter_large(Bucket B, int S)
{
    const int T = blockDim.x, n = B.n;
    const LargeView V = large_view(T);
    const LargeLane l = large_lane(B, S);
    double mi, x[3], v[3], a[3];
    large_load_rows(B, l, mi, x, v, a);
    V.m[l.tid] = mi;
    const double one[3] = {mi, 0.0, 0.0};
    double Ms[3], st[3], sx[3], x0[3], sv[3], v0[3];
    large_sys_wsum3(V, T, l, n, 0, 1.0, one, Ms, st);
    large_sys_wsum3(V, T, l, n, 0, mi, x, sx, x0);
    large_sys_wsum3(V, T, l, n, 0, mi, v, sv, v0);
    const double M = Ms[0];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double X = sx[c] / M, Vc = sv[c] / M;
        if (l.b == 0) {
            x[c] = X;
            v[c] = Vc;
        } else {
            x[c] -= x0[c];
            v[c] -= Vc;
        }
    }
    large_mvs_acc(V, l, n, x, a);
    large_store_rows(B, l, x, v, a, true);
}

// MVS form -> inertial of a bucket (from_mvs); the a0 rows are left as they are.
__global__ __launch_bounds__(kLargeMaxLanes) void k_mvs_leave_large(Bucket B, int S)
{
    const int T = blockDim.x;
    const LargeView V = large_view(T);
    const LargeLane l = large_lane(B, S);
    double mi, x[3], v[3], a[3];
    large_load_rows(B, l, mi, x, v, a);
    V.m[l.tid] = mi;
    large_from_mvs(V, T, l, B.n, mi, x, v);
    large_store_rows(B, l, x, v, a, false);
}

// Fixed-step MVS integration, one body per lane, for at most P.quantum steps
// (the clock of the Hermite kernels; the steps of mvs_step, with the
// outcomes of a system predicating its updates).  WAVES is the waves per
// SIMD the register allocator targets: 2 (unspilled) for systems of up to 16
// bodies, 4 (a few VGPRs spilled, twice the waves to hide the Kepler
// solver's latency) for larger ones, where it measured 16-23% faster.
template <int WAVES>
__global__ __launch_bounds__(kLargeMaxLanes) __attribute__((amdgpu_waves_per_eu(WAVES)))
void k_plain_mvs_large(Bucket B, StepParams P, int S)
{
    const int T = blockDim.x, n = B.n;
    const LargeView V = large_view(T);
    const LargeLane l = large_lane(B, S);
    const bool planet = l.b > 0;
    double mi, Q[3], W[3], acc[3];
    large_load_rows(B, l, mi, Q, W, acc);
    V.m[l.tid] = mi;
    Clock c;
    c.status = ST_DONE;
    if (l.valid)
        c = load_clock(B, l.slot);
    __syncthreads();
    const double m0 = l.valid ? V.m[l.base] : 1.0;
    const double inv_m0 = 1.0 / m0;
    // drift of Q (planets) by h sum_j m_j V_j / m0 and of X (star) by h Vc
    auto drift = [&](const bool on, const double h) {
        double Pm[3], unused[3];
        large_sys_wsum3(V, T, l, n, 1, mi, W, Pm, unused);
        if (!on)
            return;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (planet)
                Q[k] += h * Pm[k] * inv_m0;
            else
                Q[k] = fma(h, W[k], Q[k]);
        }
    };
    for (int q = 0; q < P.quantum; ++q) {
        double h = 0.0;
        bool last = false;
        const bool act = l.valid && plan_step(c, P, h, last);
        if (!__syncthreads_or(act))
            break;
        const double hh = 0.5 * h;
        drift(act, hh);
        if (act && planet)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                W[k] = fma(hh, acc[k], W[k]);
        int unbound = 0;
        if (act && planet) {
            const double r2 = fma(Q[2], Q[2], fma(Q[1], Q[1], Q[0] * Q[0]));
            const double v2 = fma(W[2], W[2], fma(W[1], W[1], W[0] * W[0]));
            unbound = (2.0 / sqrt(r2) - v2 / m0 > 0.0) ? 0 : 1;
        }
        const int unbound_sys = large_sys_or(V, l, n, unbound);   // every lane: barriers inside
        const bool undo = act && unbound_sys;
        if (undo && planet)
#pragma unroll
            for (int k = 0; k < 3; ++k)
                W[k] = fma(-hh, acc[k], W[k]);
        drift(undo, -hh);
        const bool go = act && !undo;
        const int kfail = (go && planet && !kepler_drift(m0, Q, W, h)) ? 1 : 0;
        const int kfail_sys = large_sys_or(V, l, n, kfail);       // every lane: barriers inside
        const bool failed = go && kfail_sys;
        const bool ok = go && !failed;
        double an[3];
        large_mvs_acc(V, l, n, Q, an);
        if (ok && planet)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                acc[k] = an[k];
                W[k] = fma(hh, acc[k], W[k]);
            }
        drift(ok, hh);
        if (ok)
            finish_step(c, P, last, h, 0.0);
        if (undo || failed)
            c.status = ST_UNBOUND;
    }
    const int bad = large_sys_or(V, l, n, (l.valid && !(finite3(Q) && finite3(W))) ? 1 : 0);
    if (!l.valid)
        return;
    if (bad)
        c.status = ST_NONFINITE;
    large_store_rows(B, l, Q, W, acc, true);
    if (l.b == 0)
        store_clock(B, l.slot, c);
}

// State read-back of a bucket in MVS form, converted to inertial (x, v) on
// the way out (the layouts of k_unpack).
__global__ __launch_bounds__(kLargeMaxLanes) void k_unpack_mvs_large(
    Bucket B, int S, const long long *__restrict__ orig_off, double *pos, double *vel, double *t,
    int *status, long long *steps)
{
    const int T = blockDim.x;
    const LargeView V = large_view(T);
    const LargeLane l = large_lane(B, S);
    double mi, x[3], v[3], a[3];
    large_load_rows(B, l, mi, x, v, a);
    V.m[l.tid] = mi;
    large_from_mvs(V, T, l, B.n, mi, x, v);
    if (!l.valid)
        return;
    const int o = B.orig[l.slot];
    const long long base = orig_off[o];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const size_t row = 3 * (base + l.b) + c;
        if (pos) pos[row] = x[c];
        if (vel) vel[row] = v[c];
    }
    if (l.b == 0) {
        if (t) t[o] = B.t[l.slot];
        if (status) status[o] = B.status[l.slot];
        if (steps) steps[o] = B.steps[l.slot];
    }
}

// ---------------------------------------------------------------------------
// Runge-Kutta Cash-Karp for large systems (n > 16): one body per lane across
// a workgroup
// ---------------------------------------------------------------------------
// The stages, weights and error control of k_plain_rkck in the large-n
// layout.  Each stage's positions go to one of two LDS copies in turn, so a
// stage costs one workgroup barrier; a body's own term is an exact zero
// through the r^2 floor, so every lane runs the same partner loop (planets in
// ascending order, the star last).

// Acceleration of this lane's body (Eq. 1) at the stage positions xs,
// published in copy cp.
__device__ __forceinline__ void large_rk_accel(const LargeView &V, const int T, const int cp,
                                               const LargeLane &l, const int n,
                                               const double (&xs)[3], double (&acc)[3])
{
    double2 *xy = V.xy + cp * T, *zvx = V.zvx + cp * T;
    xy[l.tid] = make_double2(xs[0], xs[1]);
    zvx[l.tid] = make_double2(xs[2], 0.0);
    __syncthreads();
    acc[0] = acc[1] = acc[2] = 0.0;
    if (!l.valid)
        return;
    for (int k = 1; k <= n; ++k) {
        const int j = k < n ? k : 0;   // planets 1..n-1, then the star
        const double2 p0 = xy[l.base + j], p1 = zvx[l.base + j];
        const double rx = p0.x - xs[0], ry = p0.y - xs[1], rz = p1.x - xs[2];
        const double ri = rsqrt_nr(fmax(fma(rz, rz, fma(ry, ry, rx * rx)), kLargeMinR2));
        const double mr3 = V.m[l.base + j] * (ri * ri * ri);
        acc[0] = fma(mr3, rx, acc[0]);
        acc[1] = fma(mr3, ry, acc[1]);
        acc[2] = fma(mr3, rz, acc[2]);
    }
}

// Maximum of one value per lane over the lane's system, to every valid lane.
__device__ __forceinline__ double large_sys_max(const LargeView &V, const LargeLane &l,
                                                const int n, const double v)
{
    V.red[l.tid] = v;
    __syncthreads();
    double r = 0.0;
    if (l.valid) {
        r = V.red[l.base];
        for (int b = 1; b < n; ++b)
            r = fmax(r, V.red[l.base + b]);
    }
    __syncthreads();
    return r;
}

template <bool ADV>
__global__ __launch_bounds__(kLargeMaxLanes) void k_plain_rkck_large(Bucket B, StepParams P,
                                                                     double eps, int S)
{
    using Tb = RkTableau;
    const int T = blockDim.x, n = B.n;
    const LargeView V = large_view(T);
    const LargeLane l = large_lane(B, S);
    const size_t pitch = B.pitch;
    double mi = 0.0, x[3] = {0.0, 0.0, 0.0}, v[3] = {0.0, 0.0, 0.0};
    Clock c;
    c.status = ST_DONE;
    if (l.valid) {
        mi = B.st[(R_M * n + l.b) * pitch + l.slot];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            x[cc] = B.st[((R_X + cc) * n + l.b) * pitch + l.slot];
            v[cc] = B.st[((R_V + cc) * n + l.b) * pitch + l.slot];
        }
        c = load_clock(B, l.slot);
    }
    V.m[l.tid] = mi;   // ordered before any read by the loop's first barrier
    int cp = 0;
    for (int q = 0; q < P.quantum; ++q) {
        double h = 0.0;
        bool last = false;
        const bool act = l.valid && plan_step(c, P, h, last);
        if (!__syncthreads_or(act))
            break;
        if (!act)
            h = 0.0;
        double kx[6][3], kv[6][3];
#pragma unroll
        for (int st = 0; st < 6; ++st) {
            double xs[3];
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                double dx = 0.0, dv = 0.0;
#pragma unroll
                for (int j = 0; j < st; ++j) {
                    dx = fma(Tb::a[st][j], kx[j][cc], dx);
                    dv = fma(Tb::a[st][j], kv[j][cc], dv);
                }
                xs[cc] = fma(h, dx, x[cc]);
                kx[st][cc] = fma(h, dv, v[cc]);
            }
            large_rk_accel(V, T, cp, l, n, xs, kv[st]);
            cp ^= 1;
        }
        double x5[3], v5[3], ex[3], ev[3];
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) {
            double sx = 0.0, sv = 0.0, ux = 0.0, uv = 0.0;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                sx = fma(Tb::b[j], kx[j][cc], sx);
                sv = fma(Tb::b[j], kv[j][cc], sv);
                ux = fma(Tb::e[j], kx[j][cc], ux);
                uv = fma(Tb::e[j], kv[j][cc], uv);
            }
            x5[cc] = fma(h, sx, x[cc]);
            v5[cc] = fma(h, sv, v[cc]);
            ex[cc] = h * ux;
            ev[cc] = h * uv;
        }
        bool accept = true;
        double dtp = 0.0;
        if (ADV) {
            const double X = large_sys_max(V, l, n, norm3d(x));
            const double Vm = large_sys_max(V, l, n, norm3d(v));
            const double E = large_sys_max(V, l, n, fmax(norm3d(ex) / (eps * X), norm3d(ev) / (eps * Vm)));
            accept = E <= 1.0;
            if (act && !accept) {
                if (!__builtin_isfinite(E))
                    c.status = ST_NONFINITE;
                else
                    c.dtn = h * fmax(0.1, 0.9 * pow(E, -0.25));
            }
            dtp = last ? c.dtn : h * (E > 0.0 ? fmin(5.0, fmax(0.2, 0.9 * pow(E, -0.2))) : 5.0);
        }
        if (act && accept) {
#pragma unroll
            for (int cc = 0; cc < 3; ++cc) {
                x[cc] = x5[cc];
                v[cc] = v5[cc];
            }
            finish_step(c, P, last, h, dtp);
        }
    }
    const int bad = ADV ? 0 : large_sys_or(V, l, n, (l.valid && !(finite3(x) && finite3(v))) ? 1 : 0);
    if (!l.valid)
        return;
    if (bad)
        c.status = ST_NONFINITE;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
        B.st[((R_X + cc) * n + l.b) * pitch + l.slot] = x[cc];
        B.st[((R_V + cc) * n + l.b) * pitch + l.slot] = v[cc];
    }
    if (l.b == 0)
        store_clock(B, l.slot, c);
}

// FP64 issue-ceiling probe for the roofline: each lane runs kFmaChains
// independent FMA chains (a <- a*b + c, b slightly below 1 so values stay
// bounded), so the rate is set by VALU issue rather than FMA latency.
constexpr int kFmaChains = 16;

__global__ __launch_bounds__(256) void k_fma_probe(double *out, int iters, double b, double c)
{
    double acc[kFmaChains];
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k)
        acc[k] = 1e-3 * threadIdx.x + k;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kFmaChains; ++k)
            acc[k] = fma(acc[k], b, c);
    }
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k)
        sum += acc[k];
    out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = sum;
}

inline dim3 grid_for(int n, int block) { return dim3((unsigned)((n + block - 1) / block)); }

// The device reciprocal square root of every pair evaluation, elementwise
// over n values (a check of its accuracy against a correctly rounded
// reference).
__global__ void k_rsqrt(const double *__restrict__ in, double *__restrict__ out, long long n)
{
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        out[i] = rsqrt_nr(in[i]);
}

// Checkpoint restore: the carried (a0, j0) rows and each system's clock
// (adaptive step, steps since creation, status) from caller-order arrays.
// Positions, velocities, masses and t were packed already.
__global__ void k_restore(Bucket B, const long long *__restrict__ orig_off,
                          const double *__restrict__ acc, const double *__restrict__ jerk,
                          const double *__restrict__ dtn, const long long *__restrict__ steps,
                          const int *__restrict__ status)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= B.count)
        return;
    const size_t pitch = B.pitch;
    const int n = B.n;
    const int o = B.orig[s];
    const long long base = orig_off[o];
    for (int b = 0; b < n; ++b)
        for (int c = 0; c < 3; ++c) {
            const size_t row = 3 * (base + b) + c;
            B.st[((R_A + c) * n + b) * pitch + s] = acc[row];
            B.st[((R_J + c) * n + b) * pitch + s] = jerk[row];
        }
    B.dtn[s] = dtn[o];
    B.steps[s] = steps[o];
    B.status[s] = status[o];
}

// Tables of a single homogeneous bucket whose slots are the caller's
// systems in order: slot -> system (padding slots -> 0), body offsets
// o * n, and the input-check flag cleared.
__global__ void k_identity_tables(Bucket B, long long *__restrict__ orig_off, int *bad)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < B.pitch)
        B.orig[s] = s < B.count ? s : 0;
    if (s <= B.count)
        orig_off[s] = (long long)s * B.n;
    if (s == 0)
        *bad = 0;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define FB_SWITCH_N(n, MACRO)                                                           \
    switch (n) {                                                                        \
    case 2: MACRO(2); break;  case 3: MACRO(3); break;  case 4: MACRO(4); break;        \
    case 5: MACRO(5); break;  case 6: MACRO(6); break;  case 7: MACRO(7); break;        \
    case 8: MACRO(8); break;  case 9: MACRO(9); break;  case 10: MACRO(10); break;      \
    case 11: MACRO(11); break; case 12: MACRO(12); break; case 13: MACRO(13); break;    \
    case 14: MACRO(14); break; case 15: MACRO(15); break; case 16: MACRO(16); break;    \
    default: return hipErrorInvalidValue;                                               \
    }

hipError_t launch_pack(const Bucket &B, const double *mass, const double *pos,
                       const double *vel, const double *t0, const long long *orig_off, int *bad,
                       bool pad_tail, hipStream_t s)
{
    const int limit = pad_tail ? B.pitch : B.count;
    if (limit == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_pack, grid_for(limit, 256), dim3(256), 0, s, B, mass, pos, vel, t0,
                       orig_off, bad, limit);
    return hipGetLastError();
}

void large_shape(int n, int k, int &T, int &S)
{
    T = 0;
    S = 0;
    if (k < 1)
        return;
    const int H = (n + k - 1) / k;   // lanes per system
    long long best_used = -1, best_T = 1;
    for (int t = 64; t <= kLargeMaxLanes / k; t += 64) {
        const int s = t / H;
        if (s < 1)
            continue;
        // more of the lanes in use (s H / t), compared exactly; ties keep the smaller t
        if ((long long)s * H * best_T > best_used * t) {
            best_used = (long long)s * H;
            best_T = t;
            T = t;
            S = s;
        }
    }
}

int large_bodies_per_lane(int n)
{
    // Two bodies per lane halve the LDS reads per interaction; one is kept
    // where pairing would idle clearly more body slots (odd n with few
    // systems per workgroup).
    int T1, S1, T2, S2;
    large_shape(n, 1, T1, S1);
    large_shape(n, 2, T2, S2);
    if (S2 < 1)
        return 1;
    if (S1 < 1)
        return 2;
    const double use1 = (double)S1 * n / T1, use2 = (double)S2 * n / (2.0 * T2);
    return use2 >= use1 - 0.02 ? 2 : 1;
}

namespace {
// Launch geometry of a large-n bucket with k bodies per lane: grid, lanes,
// systems per workgroup.
bool large_launch(const Bucket &B, int k, dim3 &grid, int &T, int &S)
{
    large_shape(B.n, k, T, S);
    if (S < 1)
        return false;
    grid = dim3((unsigned)((B.count + S - 1) / S));
    return true;
}
}  // namespace

hipError_t launch_prepare(const Bucket &B, hipStream_t s)
{
    if (B.count == 0)
        return hipSuccess;
    if (B.n > kMaxBodies) {
        dim3 grid;
        int T, S;
        if (!large_launch(B, 1, grid, T, S))
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_prepare_large, grid, dim3(T), large_lds_bytes(T), s, B, S);
        return hipGetLastError();
    }
#define FB_L(NN) hipLaunchKernelGGL(k_prepare<NN>, grid_for(B.count, 64), dim3(64), 0, s, B)
    FB_SWITCH_N(B.n, FB_L)
#undef FB_L
    return hipGetLastError();
}

hipError_t launch_begin_run(const Bucket &B, int fixed_steps, long long n_steps, double t_end,
                            double dt, int adaptive, double eta, hipStream_t s)
{
    if (B.count == 0)
        return hipSuccess;
    if (B.n > kMaxBodies) {
        dim3 grid;
        int T, S;
        if (!large_launch(B, 1, grid, T, S))
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_begin_run_large, grid, dim3(T), large_lds_bytes(T), s, B, S,
                           fixed_steps, n_steps, t_end, dt, adaptive, eta);
        return hipGetLastError();
    }
#define FB_L(NN)                                                                        \
    hipLaunchKernelGGL(k_begin_run<NN>, grid_for(B.count, 64), dim3(64), 0, s, B,       \
                       fixed_steps, n_steps, t_end, dt, adaptive, eta)
    FB_SWITCH_N(B.n, FB_L)
#undef FB_L
    return hipGetLastError();
}

hipError_t launch_plain(const Bucket &B, int mapping, int waves_per_group, const StepParams &P,
                        hipStream_t s)
{
    if (B.count == 0)
        return hipSuccess;
    const int W = waves_per_group < 1 ? 1 : (waves_per_group > 4 ? 4 : waves_per_group);
    const bool adv = P.adaptive || P.stop_rules;
    if (B.n > kMaxBodies) {
        dim3 grid;
        int T, S;
        const int K = large_bodies_per_lane(B.n);
        if (!large_launch(B, K, grid, T, S))
            return hipErrorInvalidValue;
        const size_t lds = large_lds_bytes(K * T);
        if (K == 2 && adv)
            hipLaunchKernelGGL((k_plain_large<2, true>), grid, dim3(T), lds, s, B, P, S);
        else if (K == 2)
            hipLaunchKernelGGL((k_plain_large<2, false>), grid, dim3(T), lds, s, B, P, S);
        else if (adv)
            hipLaunchKernelGGL((k_plain_large<1, true>), grid, dim3(T), lds, s, B, P, S);
        else
            hipLaunchKernelGGL((k_plain_large<1, false>), grid, dim3(T), lds, s, B, P, S);
        return hipGetLastError();
    }
    if (mapping == MAP_SPL && B.n <= (adv ? kMaxSplAdv : kMaxSplBodies)) {
        const dim3 grid = grid_for(B.count, 64 * W);
#define FB_LA(NN)                                                                       \
    hipLaunchKernelGGL((k_plain_spl<NN, true>), grid, dim3(64 * W), spl_lds_bytes(NN) * W, \
                       s, B, P)
#define FB_LF(NN)                                                                       \
    hipLaunchKernelGGL((k_plain_spl<NN, false>), grid, dim3(64 * W), spl_lds_bytes(NN) * W, \
                       s, B, P)
        if (adv) {
            switch (B.n) {
            case 2: FB_LA(2); break;
            case 3: FB_LA(3); break;
            case 4: FB_LA(4); break;
            case 5: FB_LA(5); break;
            case 6: FB_LA(6); break;
            case 7: FB_LA(7); break;
            case 8: FB_LA(8); break;
            default: return hipErrorInvalidValue;
            }
        } else {
            switch (B.n) {
            case 2: FB_LF(2); break;
            case 3: FB_LF(3); break;
            case 4: FB_LF(4); break;
            case 5: FB_LF(5); break;
            case 6: FB_LF(6); break;
            case 7: FB_LF(7); break;
            case 8: FB_LF(8); break;
            case 9: FB_LF(9); break;
            case 10: FB_LF(10); break;
            default: return hipErrorInvalidValue;
            }
        }
#undef FB_LA
#undef FB_LF
        return hipGetLastError();
    }
    const int S = 64 / B.n;
    const int tiles = (B.count + S - 1) / S;
    const dim3 grid((unsigned)((tiles + W - 1) / W));
    const size_t lds = sizeof(BplLds) * W;
#define FB_L(NN)                                                                           \
    if (adv) hipLaunchKernelGGL((k_plain_bpl<NN, true>), grid, dim3(64 * W), lds, s, B, P);  \
    else hipLaunchKernelGGL((k_plain_bpl<NN, false>), grid, dim3(64 * W), lds, s, B, P)
    FB_SWITCH_N(B.n, FB_L)
#undef FB_L
    return hipGetLastError();
}

size_t persistent_lds_bytes(int spl_class, int waves_per_group)
{
    const size_t per_wave = spl_class ? kWideLdsStride : sizeof(BplLds);
    return per_wave * waves_per_group;
}

int persistent_max_groups_per_cu(int adv, int spl_class, int waves_per_group)
{
    int blocks = 0;
    const int threads = 64 * waves_per_group;
    const size_t lds = persistent_lds_bytes(spl_class, waves_per_group);
    hipError_t e;
    if (spl_class)
        e = adv ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_persistent_spl<true, true>,
                                                               threads, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_persistent_spl<false, false>,
                                                               threads, lds);
    else
        e = adv ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_persistent<true, true>,
                                                               threads, lds)
                : hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_persistent<false, false>,
                                                               threads, lds);
    return e == hipSuccess ? blocks : 0;
}

hipError_t launch_persistent(const Bucket *d_buckets, const Tile *d_tiles, const int *d_ntiles,
                             int *d_head, const int *d_lists, const StepParams &P, int adv,
                             int spl_class, int grid, int waves_per_group, ActiveLists *compact,
                             hipStream_t s)
{
    const int W = waves_per_group < 1 ? 1 : (waves_per_group > 4 ? 4 : waves_per_group);
    const size_t lds = persistent_lds_bytes(spl_class, W);
    ActiveLists AL = compact ? *compact : ActiveLists{nullptr, nullptr, nullptr, nullptr, nullptr};
    const dim3 g(grid), b(64 * W);
#define FB_P(KERNEL, A, C)                                                               \
    hipLaunchKernelGGL((KERNEL<A, C>), g, b, lds, s, d_buckets, d_tiles, d_ntiles, d_head, \
                       d_lists, P, AL)
    if (spl_class) {
        if (adv) {
            if (compact) FB_P(k_persistent_spl, true, true); else FB_P(k_persistent_spl, true, false);
        } else {
            if (compact) FB_P(k_persistent_spl, false, true); else FB_P(k_persistent_spl, false, false);
        }
    } else {
        if (adv) {
            if (compact) FB_P(k_persistent, true, true); else FB_P(k_persistent, true, false);
        } else {
            if (compact) FB_P(k_persistent, false, true); else FB_P(k_persistent, false, false);
        }
    }
#undef FB_P
    return hipGetLastError();
}

hipError_t launch_build_tiles(const Bucket *d_buckets, int n_buckets, const int *d_order,
                              const int *d_mapping, ActiveLists L, Tile *d_tiles, int *d_ntiles,
                              int *d_head, hipStream_t s)
{
    if (n_buckets < 0 || n_buckets > kMaxBodies + 1)   // the kernel's tables hold kMaxBodies + 2
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_build_tiles, dim3(1), dim3(256), 0, s, d_buckets, n_buckets, d_order,
                       d_mapping, L, d_tiles, d_ntiles, d_head);
    return hipGetLastError();
}

hipError_t launch_reset_counter(int *p, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_int, grid_for(n, 256), dim3(256), 0, s, p, n, 0);
    return hipGetLastError();
}

hipError_t launch_unpack(const Bucket &B, const long long *orig_off, double *pos, double *vel,
                         double *acc, double *jerk, double *t, int *status, long long *steps,
                         double *dt_next, hipStream_t s)
{
    if (B.count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_unpack, grid_for(B.count, 256), dim3(256), 0, s, B, orig_off, pos, vel,
                       acc, jerk, t, status, steps, dt_next);
    return hipGetLastError();
}

hipError_t launch_diag(const Bucket &B, double *energy, double *angmom, bool mvs_form,
                       hipStream_t s)
{
    if (B.count == 0)
        return hipSuccess;
    if (B.n > kMaxBodies || (mvs_form && B.n > kMaxMvsBodies)) {
        dim3 grid;
        int T, S;
        if (!large_launch(B, 1, grid, T, S))
            return hipErrorInvalidValue;
        if (mvs_form)
            hipLaunchKernelGGL(k_diag_large<true>, grid, dim3(T), large_lds_bytes(T), s, B, S,
                               energy, angmom);
        else
            hipLaunchKernelGGL(k_diag_large<false>, grid, dim3(T), large_lds_bytes(T), s, B, S,
                               energy, angmom);
        return hipGetLastError();
    }
    if (mvs_form) {
        if (B.n > kMaxMvsBodies)
            return hipErrorInvalidValue;
#define FB_L(NN) hipLaunchKernelGGL((k_diag<NN, true>), grid_for(B.count, 64), dim3(64), 0, s, B, energy, angmom)
        FB_SWITCH_N(B.n, FB_L)
#undef FB_L
    } else {
#define FB_L(NN) hipLaunchKernelGGL((k_diag<NN, false>), grid_for(B.count, 64), dim3(64), 0, s, B, energy, angmom)
        FB_SWITCH_N(B.n, FB_L)
#undef FB_L
    }
    return hipGetLastError();
}

#define FB_SWITCH_MVS(n, MACRO)                                                         \
    switch (n) {                                                                        \
    case 2: MACRO(2); break;  case 3: MACRO(3); break;  case 4: MACRO(4); break;        \
    case 5: MACRO(5); break;  case 6: MACRO(6); break;  case 7: MACRO(7); break;        \
    case 8: MACRO(8); break;                                                            \
    default: return hipErrorInvalidValue;                                               \
    }
static_assert(kMaxMvsBodies == 8, "FB_SWITCH_MVS covers n = 2..kMaxMvsBodies");

hipError_t launch_mvs_enter(const Bucket &B, hipStream_t s)
{
    if (B.count == 0)
        return hipSuccess;
    if (B.n > kMaxMvsBodies) {
        dim3 grid;
        int T, S;
        if (!large_launch(B, 1, grid, T, S))
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_mvs_enter_large, grid, dim3(T), large_lds_bytes(T), s, B, S);
        return hipGetLastError();
    }
#define FB_L(NN) hipLaunchKernelGGL(k_mvs_enter<NN>, grid_for(B.count, 64), dim3(64), 0, s, B)
    FB_SWITCH_MVS(B.n, FB_L)
#undef FB_L
    return hipGetLastError();
}

hipError_t launch_mvs_leave(const Bucket &B, hipStream_t s)
{
    if (B.count == 0)
        return hipSuccess;
    if (B.n > kMaxMvsBodies) {
        dim3 grid;
        int T, S;
        if (!large_launch(B, 1, grid, T, S))
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_mvs_leave_large, grid, dim3(T), large_lds_bytes(T), s, B, S);
        return hipGetLastError();
    }
#define FB_L(NN) hipLaunchKernelGGL(k_mvs_leave<NN>, grid_for(B.count, 64), dim3(64), 0, s, B)
    FB_SWITCH_MVS(B.n, FB_L)
#undef FB_L
    return hipGetLastError();
}

hipError_t launch_plain_mvs(const Bucket &B, int mapping, int waves_per_group, const StepParams &P,
                            hipStream_t s)
{
    if (B.count == 0)
        return hipSuccess;
    if (B.n > kMaxMvsBodies || mapping != MAP_SPL) {
        dim3 lgrid;
        int T, S;
        if (!large_launch(B, 1, lgrid, T, S))
            return hipErrorInvalidValue;
        if (B.n > kMaxBodies)
            hipLaunchKernelGGL(k_plain_mvs_large<4>, lgrid, dim3(T), large_lds_bytes(T), s, B, P, S);
        else
            hipLaunchKernelGGL(k_plain_mvs_large<2>, lgrid, dim3(T), large_lds_bytes(T), s, B, P, S);
        return hipGetLastError();
    }
    const int W = waves_per_group < 1 ? 1 : (waves_per_group > 4 ? 4 : waves_per_group);
    const dim3 grid = grid_for(B.count, 64 * W);
#define FB_L(NN) hipLaunchKernelGGL(k_plain_mvs<NN>, grid, dim3(64 * W), 0, s, B, P)
    FB_SWITCH_MVS(B.n, FB_L)
#undef FB_L
    return hipGetLastError();
}

hipError_t launch_unpack_mvs(const Bucket &B, const long long *orig_off, double *pos, double *vel,
                             double *t, int *status, long long *steps, hipStream_t s)
{
    if (B.count == 0)
        return hipSuccess;
    if (B.n > kMaxMvsBodies) {
        dim3 grid;
        int T, S;
        if (!large_launch(B, 1, grid, T, S))
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_unpack_mvs_large, grid, dim3(T), large_lds_bytes(T), s, B, S, orig_off,
                           pos, vel, t, status, steps);
        return hipGetLastError();
    }
#define FB_L(NN) hipLaunchKernelGGL(k_unpack_mvs<NN>, grid_for(B.count, 64), dim3(64), 0, s, B, \
                                    orig_off, pos, vel, t, status, steps)
    FB_SWITCH_MVS(B.n, FB_L)
#undef FB_L
    return hipGetLastError();
}

hipError_t launch_count_active(const Bucket &B, int *count, hipStream_t s)
{
    if (B.count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_count_active, grid_for(B.count, 256), dim3(256), 0, s, B, count);
    return hipGetLastError();
}

hipError_t launch_log(const Bucket &B, const long long *orig_off, int kind, const double *los,
                      int k, int max_records, double *out, hipStream_t s)
{
    if (B.count == 0)
        return hipSuccess;
    if (B.n > kMaxBodies) {
        dim3 grid;
        int T, S;
        if (!large_launch(B, 1, grid, T, S))
            return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_log_large, grid, dim3(T), large_lds_bytes(T), s, B, S, orig_off,
                           kind, los[0], los[1], los[2], k, max_records, out);
        return hipGetLastError();
    }
#define FB_L(NN) hipLaunchKernelGGL(k_log<NN>, grid_for(B.count, 64), dim3(64), 0, s, B, orig_off, \
                                    kind, los[0], los[1], los[2], k, max_records, out)
    FB_SWITCH_N(B.n, FB_L)
#undef FB_L
    return hipGetLastError();
}

hipError_t launch_plain_rkck(const Bucket &B, int waves_per_group, const StepParams &P,
                             double eps, hipStream_t s)
{
    if (B.count == 0)
        return hipSuccess;
    if (B.n > kMaxBodies) {
        dim3 grid;
        int T, S;
        if (!large_launch(B, 1, grid, T, S))
            return hipErrorInvalidValue;
        if (P.adaptive)
            hipLaunchKernelGGL(k_plain_rkck_large<true>, grid, dim3(T), large_lds_bytes(T), s, B, P,
                               eps, S);
        else
            hipLaunchKernelGGL(k_plain_rkck_large<false>, grid, dim3(T), large_lds_bytes(T), s, B,
                               P, eps, S);
        return hipGetLastError();
    }
    const int W = waves_per_group < 1 ? 1 : (waves_per_group > 4 ? 4 : waves_per_group);
    const int S = 64 / B.n;
    const int tiles = (B.count + S - 1) / S;
    const dim3 grid((unsigned)((tiles + W - 1) / W));
    const size_t lds = sizeof(BplLds) * W;
    if (eps > 0.0) {
#define FB_L(NN) hipLaunchKernelGGL((k_plain_rkck<NN, true>), grid, dim3(64 * W), lds, s, B, P, eps)
        FB_SWITCH_N(B.n, FB_L)
#undef FB_L
    } else {
#define FB_L(NN) hipLaunchKernelGGL((k_plain_rkck<NN, false>), grid, dim3(64 * W), lds, s, B, P, eps)
        FB_SWITCH_N(B.n, FB_L)
#undef FB_L
    }
    return hipGetLastError();
}

hipError_t launch_fma_probe(double *out, int blocks, int iters, hipStream_t s)
{
    hipLaunchKernelGGL(k_fma_probe, dim3(blocks), dim3(256), 0, s, out, iters, 0.999999, 1e-6);
    return hipGetLastError();
}

hipError_t launch_rsqrt(const double *in, double *out, long long n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const long long blocks = (n + 255) / 256;
    if (blocks > INT_MAX)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_rsqrt, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_restore(const Bucket &B, const long long *orig_off, const double *acc,
                          const double *jerk, const double *dtn, const long long *steps,
                          const int *status, hipStream_t s)
{
    if (B.count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_restore, grid_for(B.count, 256), dim3(256), 0, s, B, orig_off, acc, jerk,
                       dtn, steps, status);
    return hipGetLastError();
}

hipError_t launch_identity_tables(const Bucket &B, long long *orig_off, int *bad, hipStream_t s)
{
    hipLaunchKernelGGL(k_identity_tables, grid_for(B.pitch + 1, 256), dim3(256), 0, s, B,
                       orig_off, bad);
    return hipGetLastError();
}

}  // namespace fb
