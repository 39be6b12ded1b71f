/*
 * fewbody.h -- C ABI of libfewbody: FP64 fourth-order time-symmetrised
 * Hermite P(EC)^2 integration of very many independent few-body systems on
 * one AMD MI355X (gfx950).
 *
 * The method is the Hermite predictor-corrector of the Swarm-NG paper
 * (arXiv:1208.1157): Newtonian pair acceleration with G = 1 (Section 2.1,
 * Eq. 1) and its analytic time derivative (the jerk, Section 2.2.1), the
 * predictor of Eq. 3, the corrector of Eq. 4 applied twice per step
 * (Algorithm 2), inside the many-steps-per-launch loop of Algorithm 1.
 * Eq. 4 is read with coefficient 3/20, a (dt)^3 jerk term and the predicted
 * state as the base of every correction; the step's last evaluation is
 * carried as the next step's (a0, j0).
 *
 * Conventions shared by every call
 * --------------------------------
 * Ensembles are ragged: system s has n_body[s] bodies (2..FB_MAX_BODIES);
 * body 0 of each system is its central star (only the stop rules care).
 * Systems of up to FB_MAX_SMALL_BODIES bodies run kernels specialised per
 * body count.  Larger ones run the large-n gravitation (Section 4.2's second
 * variant: one body per lane across a workgroup, each pair evaluated from
 * both sides): Hermite steps, fixed or adaptive, with stop rules, monitors
 * and diagnostics; on the persistent schedule they run as plain launches
 * inside every quantum, beside the fused launch of the smaller systems.
 * MVS and Runge-Kutta run them too; the autotuner leaves their launch shape
 * alone (it tunes the other buckets and the persistent launch around them);
 * the server rejects them with FB_E_INVAL.
 * Flat body arrays are body-major: body b of system s is row off[s] + b with
 * off the exclusive prefix sum of n_body; pos/vel/acc/jerk rows hold x,y,z.
 * All floating point is IEEE binary64.
 *
 * Errors: every call returns an fb_status; FB_OK is 0 and every error is
 * negative.  fb_last_error() returns a thread-local message for the most
 * recent failure.  No C++ exception crosses this interface.
 *
 * Ownership: the caller keeps every buffer it passes; the library copies
 * inputs during the call and never frees or retains caller memory, except
 * the workspace of fb_ensemble_create_device, which must outlive the
 * ensemble.  Streams are borrowed (NULL = the null stream).  Work is
 * enqueued asynchronously on the ensemble's stream; fb_get_* calls and
 * fb_diagnostics synchronise that stream before they return.
 *
 * Run-time failures of a single system (non-finite state, e.g. coincident
 * bodies) mark that system's status and never fail the call.
 */
#ifndef FEWBODY_H
#define FEWBODY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FB_MAX_BODIES 512        /* bodies per system                        */
#define FB_MAX_SMALL_BODIES 16   /* ... for every integrator and schedule    */

typedef enum {
    FB_OK = 0,
    FB_E_INVAL = -1,     /* bad argument (message says which)               */
    FB_E_NOMEM = -2,     /* device allocation failed / workspace too small  */
    FB_E_DEVICE = -3,    /* HIP runtime error                               */
    FB_E_BUDGET = -4,    /* serving: request exceeds the server's budget    */
    FB_E_STATE = -5,     /* call not valid in the object's current state    */
    FB_E_NOTFOUND = -6   /* serving: unknown request id                     */
} fb_status;

/* Per-system status codes. */
enum {
    FB_SYS_ACTIVE = 0,     /* still integrating                               */
    FB_SYS_DONE = 1,       /* reached the destination time / step count       */
    FB_SYS_ENCOUNTER = 2,  /* two planets closer than one mutual Hill radius  */
    FB_SYS_EJECTED = 3,    /* a planet farther than r_eject from its star     */
    FB_SYS_NONFINITE = 4,  /* a position or velocity became NaN or infinite   */
    FB_SYS_STALLED_DT = 5, /* adaptive step fell below 1e-12 * |t_end|        */
    FB_SYS_MAXSTEPS = 6,   /* hit fb_opts.max_steps                           */
    FB_SYS_UNBOUND = 7     /* MVS: a planet's orbit about the star is not bound
                              (state of the last completed step)              */
};

/* Stop-rule bits for fb_opts.stop_rules. */
enum { FB_STOP_ENCOUNTER = 1, FB_STOP_EJECT = 2 };

/* Lane mappings of a launch plan. */
enum {
    FB_MAP_AUTO = 0,             /* chosen per bucket at launch (see plans)    */
    FB_MAP_SYSTEM_PER_LANE = 1,  /* one system per lane, all state in VGPRs    */
    FB_MAP_BODY_PER_LANE = 2     /* one body per lane, partners through LDS    */
};

/* Schedules. */
enum {
    FB_SCHED_PLAIN = 0,       /* one launch per homogeneous body-count bucket  */
    FB_SCHED_PERSISTENT = 1   /* one fused persistent launch over all buckets,
                                 tiles pulled longest-first from a queue        */
};

/* Integration options; NULL means all defaults.  Defaults: fixed step, no
 * stop rules, eta 0.01, r_eject 100, max_steps unlimited, plain schedule,
 * one quantum for the whole run, no compaction. */
typedef struct {
    int32_t adaptive;           /* 0: fixed dt.  1: per-system adaptive step
                                   dt = eta * min over pairs |a_ij|/|j_ij| of
                                   the pair's two-body relative acceleration and
                                   jerk at the step's last evaluation (the
                                   set-up evaluation for the first step).
                                   2: Eq. 5's rule, dt = eta [sum_i |j_i|^2 /
                                   |a_i|^2]^(-1/2) from the accelerations and
                                   jerks that start the step (eta is tau).
                                   Either way the final step is shortened to
                                   land on t_end.                               */
    double eta;                 /* adaptive accuracy parameter (tau for rule 2) */
    int32_t stop_rules;         /* FB_STOP_* bits, checked after every step     */
    double r_eject;             /* ejection radius from the star                */
    int64_t max_steps;          /* per-system cap on steps (<=0: unlimited)     */
    int32_t schedule;           /* FB_SCHED_*                                   */
    int32_t steps_per_quantum;  /* persistent schedule: steps per launch
                                   (<=0: whole run in one launch); with
                                   compact and the automatic fused class,
                                   once every surviving tile has a
                                   wavefront of its own, the rest of the run
                                   goes in one launch                           */
    int32_t compact;            /* persistent schedule: rebuild tiles from the
                                   still-active systems after every quantum     */
} fb_opts;

/* Fill *o with the defaults above. */
void fb_opts_default(fb_opts *o);

/* ---------------------------------------------------------------- ensembles */
typedef struct fb_ensemble fb_ensemble;

/* Create an ensemble from HOST arrays (Section 2.1's state: masses,
 * positions, velocities of every body of every system).
 *   n_sys      number of systems (>= 0)
 *   n_body     [n_sys] bodies per system, 2..FB_MAX_BODIES
 *   mass       [N] >= 0 and finite;  pos, vel [N][3] finite;  N = sum n_body
 *   t0         [n_sys] start times, or NULL for all zero
 *   hip_stream hipStream_t to enqueue on (borrowed), NULL = null stream
 * The library allocates and owns the device state.  The set-up evaluation
 * of (a0, j0) (Algorithm 1's "prepare") runs here.  Returns FB_E_INVAL on
 * bad input, FB_E_NOMEM / FB_E_DEVICE on HIP failures. */
fb_status fb_ensemble_create(int32_t n_sys, const int32_t *n_body,
                             const double *mass, const double *pos,
                             const double *vel, const double *t0,
                             void *hip_stream, fb_ensemble **out);

/* Bytes of device workspace an ensemble of this shape needs. */
size_t fb_workspace_bytes(int32_t n_sys, const int32_t *n_body);

/* Same as fb_ensemble_create, but mass/pos/vel/t0 are DEVICE pointers (t0
 * may be NULL) and all device state lives in the caller's workspace of
 * ws_bytes >= fb_workspace_bytes(...) bytes, 256-byte aligned.  The caller
 * owns the workspace (e.g. a torch tensor) and keeps it alive until
 * fb_ensemble_destroy; n_body stays a host array.  Input values are
 * validated on the device; a bad value fails the call with FB_E_INVAL. */
fb_status fb_ensemble_create_device(int32_t n_sys, const int32_t *n_body,
                                    const double *d_mass, const double *d_pos,
                                    const double *d_vel, const double *d_t0,
                                    void *d_workspace, size_t ws_bytes,
                                    void *hip_stream, fb_ensemble **out);

/* Resume from a checkpoint (the state Section 4.4 copies between host and
 * device, with what Algorithm 2 carries from one step to the next): an
 * ensemble like fb_ensemble_create's from HOST arrays, whose (a0, j0) are
 * the given acc0/jerk0 [N][3] instead of a set-up evaluation, with each
 * system's time t [n_sys] (NULL: 0), carried adaptive step dt_next [n_sys]
 * (finite, >= 0; NULL: none carried), status [n_sys] (FB_SYS_ACTIVE ..
 * FB_SYS_MAXSTEPS; NULL: FB_SYS_DONE) and steps since creation [n_sys]
 * (>= 0; NULL: 0).  With the values fb_get_state and fb_get_hermite_state
 * returned, later integration continues bitwise as the checkpointed
 * ensemble would have.  Validation and ownership as fb_ensemble_create;
 * FB_E_INVAL names the first bad value. */
fb_status fb_ensemble_restore(int32_t n_sys, const int32_t *n_body,
                              const double *mass, const double *pos,
                              const double *vel, const double *acc0,
                              const double *jerk0, const double *t,
                              const double *dt_next, const int32_t *status,
                              const int64_t *steps, void *hip_stream,
                              fb_ensemble **out);

/* Advance every active system by exactly n_steps fixed steps of size dt
 * (Algorithm 1's loop with a step count in place of a destination time;
 * each step is Algorithm 2's P(EC)^2).  dt may be negative: backward
 * integration.  Times become t_start + n_steps * dt.  o: schedule/quantum/
 * stop options (o->adaptive must be 0); NULL = defaults.  Asynchronous on
 * the ensemble's stream; FB_E_INVAL for a bad argument. */
fb_status fb_integrate_steps(fb_ensemble *e, int64_t n_steps, double dt,
                             const fb_opts *o);

/* Mixed-variable symplectic integration (Section 2.2.3) of every active
 * system by exactly n_steps fixed steps of dt (body 0 the central star;
 * one system per lane up to 8 bodies, one body per lane across a workgroup
 * for 9..FB_MAX_BODIES).  Each step is the paper's sequence of
 * sub-steps: Cartesian drift dt/2, kick dt/2, Keplerian drift dt, kick dt/2,
 * Cartesian drift dt/2, in the democratic heliocentric splitting (Duncan,
 * Levison & Lee 1998): planets follow Kepler orbits about the star (mu =
 * m0) in heliocentric positions and barycentric velocities, kicks apply the
 * planet-planet forces, and the drift is the star's reflex motion.  Kepler's
 * equation is solved by Newton iteration per planet and step.  While the
 * ensemble holds MVS state its rows keep the MVS variables (and the last
 * kick's accelerations), so quanta and calls chain without conversion;
 * fb_get_state and fb_diagnostics convert on the way out,
 * fb_get_hermite_state fails with FB_E_STATE, and the next Hermite
 * integration converts back and re-evaluates (a0, j0).  o: the quantum (o->
 * steps_per_quantum); adaptive, stop_rules and compact must be 0 and the
 * schedule plain.  A planet whose heliocentric orbit is not bound stops its
 * system with status FB_SYS_UNBOUND. */
fb_status fb_integrate_mvs(fb_ensemble *e, int64_t n_steps, double dt, const fb_opts *o);

/* ------------------------------------------------- monitors and logging */
/* A monitor that logs every system's state at regular steps into a device
 * buffer (the logging of the generic integrator, Section 4.3), optionally
 * reduced on the device before anything crosses to the host (Section 4.4's
 * data reduction: the star's radial velocity only, or energy and angular
 * momentum). */
enum { FB_LOG_STATE = 0, FB_LOG_RV = 1, FB_LOG_ENERGY = 2 };

typedef struct {
    int32_t kind;          /* FB_LOG_*                                               */
    int32_t every;         /* a record after every `every` steps (>= 1)              */
    int32_t max_records;   /* records per system the buffer holds                    */
    int32_t reserved;      /* 0                                                      */
    double los[3];         /* FB_LOG_RV: line of sight (any non-zero length)         */
    void *d_buffer;        /* DEVICE memory, caller-owned, fb_log_bytes(...) bytes   */
    size_t buffer_bytes;
} fb_log_spec;

/* Bytes of a log buffer for systems of these body counts (caller's order)
 * and max_records records each; 0 on invalid input.  Layouts (doubles,
 * system index o in the caller's order, record k):
 *   FB_LOG_STATE:  system o's block starts at max_records * (o + 6 off[o])
 *                  with off the body offsets; record k holds t, then
 *                  pos [n_o][3], then vel [n_o][3];
 *   FB_LOG_RV:     [o][k][2] = t, (v_star - v_cm) . los / |los|;
 *   FB_LOG_ENERGY: [o][k][5] = t, E (Eq. 6), L[3]. */
size_t fb_log_bytes(int32_t n_sys, const int32_t *n_body, int32_t kind, int32_t max_records);

/* fb_integrate_steps (fixed steps, plain schedule) with the monitor of `log`:
 * record 0 is the state before the first step, then one record after every
 * `every` steps and one at the end; the integration itself is identical to
 * the unlogged call.  *n_records (may be NULL) gets the records written.
 * FB_E_INVAL if the buffer is too small or holds fewer than the run's
 * records, or for the persistent schedule. */
fb_status fb_integrate_steps_logged(fb_ensemble *e, int64_t n_steps, double dt,
                                    const fb_opts *o, const fb_log_spec *log,
                                    int32_t *n_records);

/* Integration to observation times with the monitor of `log` (Section 4.3's
 * logging at the caller's times; with FB_LOG_RV, Section 4.4's radial
 * velocity reduction at each epoch).  For k = 0 .. n_times-1 in turn, every
 * system integrates to t_obs[k] with the semantics of fb_integrate (fixed dt
 * > 0 with the last step shortened, or adaptive steps; stop rules; either
 * schedule), then record k is written.  A system stopped by a rule, or
 * already at or past t_obs[k], keeps its state: its record's t says where it
 * is.  Because each run lands on its time, the step before each time is
 * shortened, so the trajectory differs from one run straight to the last
 * time.  t_obs is a host array, finite and strictly increasing; log.every
 * is ignored; log.max_records must be >= n_times.  *n_records (may be NULL)
 * gets the records written. */
fb_status fb_integrate_to_times(fb_ensemble *e, int32_t n_times, const double *t_obs, double dt,
                                const fb_opts *o, const fb_log_spec *log, int32_t *n_records);

/* Runge-Kutta Cash-Karp integration (Sections 2.2.2 and 4.3.2): the embedded
 * 4(5) pair of Cash & Karp (1990) on (x, v) with accelerations from Eq. 1,
 * six acceleration evaluations per step or trial step, one body per lane,
 * for systems of any supported size.  The step advances with the
 * fifth-order weights; the error estimate is their difference from the
 * fourth-order ones.
 * fb_integrate_rkck_steps: exactly n_steps fixed steps of dt.
 * fb_integrate_rkck: adaptive steps from each system's t to t_end, dt being
 * the first trial step (> 0) and eps (> 0) the error tolerance.  With X and V
 * the largest |x_i| and |v_i| of a system at the step's start, a trial is
 * accepted when E = max_i max(|dx_i| / (eps X), |dv_i| / (eps V)) <= 1 (dx,
 * dv the error estimate) and the next trial is h min(5, max(0.2,
 * 0.9 E^(-1/5))); otherwise it is rejected (state and time unchanged) and
 * retried with h max(0.1, 0.9 E^(-1/4)).  The last step is shortened onto
 * t_end; a step below 1e-12 |t_end| stalls the system (FB_SYS_STALLED_DT).
 * o: the quantum and max_steps; adaptive, stop_rules and compact must be 0
 * and the schedule plain.  A later Hermite integration re-evaluates (a0,
 * j0) first; fb_get_hermite_state does the same. */
fb_status fb_integrate_rkck_steps(fb_ensemble *e, int64_t n_steps, double dt, const fb_opts *o);
fb_status fb_integrate_rkck(fb_ensemble *e, double t_end, double dt, double eps,
                            const fb_opts *o);

/* Integrate every active system to t_end (Algorithm 1's destination time).
 * Fixed step (o->adaptive == 0): whole steps of dt, then one shortened step
 * that lands on t_end (skipped when the remainder is below 1e-9 |dt|); the
 * sign of dt must match t_end - t.  Adaptive: dt is ignored; forward only.
 * Systems whose status is not ACTIVE/DONE (stopped by a rule) stay put. */
fb_status fb_integrate(fb_ensemble *e, double t_end, double dt,
                       const fb_opts *o);

/* Wait for all work enqueued on the ensemble's stream (the host's wait for
 * the device before it examines results, Section 5.3). */
fb_status fb_synchronize(fb_ensemble *e);

/* Copy state to HOST arrays in the caller's system order (the device-to-host
 * ensemble copy of Section 4.4); any pointer may be NULL to skip it.
 * pos, vel [N][3]; t [n_sys]; status [n_sys] (FB_SYS_*); steps [n_sys] =
 * steps taken since creation.  Synchronises the ensemble's stream. */
fb_status fb_get_state(fb_ensemble *e, double *pos, double *vel, double *t,
                       int32_t *status, int64_t *steps);

/* Checkpoint part of the state (what Algorithm 2 carries into the next
 * step, copied to the host as Section 4.4's ensemble copies are): the
 * carried (a0, j0) of every body, [N][3] each, and each system's carried
 * adaptive step (dt_next, [n_sys]); any pointer may be NULL.  With
 * fb_get_state's outputs it is what fb_ensemble_restore takes.
 * FB_E_STATE while the ensemble holds MVS state.  Synchronises. */
fb_status fb_get_hermite_state(fb_ensemble *e, double *acc0, double *jerk0,
                               double *dt_next);

/* Energy (Eq. 6 with each pair counted once) and angular momentum about the
 * origin (sum of m x cross v) of every system, computed on the device; only
 * these 4 doubles per system cross to the HOST arrays energy [n_sys] and
 * angmom [n_sys][3] (either may be NULL). */
fb_status fb_diagnostics(fb_ensemble *e, double *energy, double *angmom);

/* Number of systems and total bodies. */
fb_status fb_ensemble_shape(const fb_ensemble *e, int32_t *n_sys, int64_t *n_bodies);

/* Wait for the ensemble's stream, then free its device state (the library's
 * own allocation; a caller workspace is left to the caller) and the handle.
 * NULL is a no-op. */
fb_status fb_ensemble_destroy(fb_ensemble *e);

/* ------------------------------------------------ stateless batch steps */
/* Bytes of device workspace fb_hermite_steps_device needs for n_sys systems
 * of n bodies; 0 on invalid input. */
size_t fb_hermite_steps_workspace_bytes(int32_t n_sys, int32_t n);

/* n_steps fixed Hermite steps of dt (Eq. 3 predictor, Eq. 4 corrector twice
 * per step, Algorithm 2; the set-up evaluation of Algorithm 1's "prepare"
 * first) of n_sys systems of n bodies (2..FB_MAX_SMALL_BODIES) held in the
 * caller's DEVICE arrays, in place: d_mass [N], d_pos and d_vel [N][3]
 * body-major, N = n_sys * n; d_status [n_sys] (may be NULL) gets each
 * system's FB_SYS_* code (FB_SYS_DONE, or FB_SYS_NONFINITE for a system
 * whose state became non-finite).  The packed state lives in the caller's
 * workspace of ws_bytes >= fb_hermite_steps_workspace_bytes(n_sys, n)
 * bytes, 256-byte aligned, which the call only borrows.  Pure stream work:
 * no host synchronisation, no allocation, no read-back, so the inputs are
 * not checked on the host (a non-finite value ends its system as
 * FB_SYS_NONFINITE).  Same kernels and plan as an ensemble's plain
 * schedule: the results equal fb_ensemble_create_device + fb_integrate_steps
 * + fb_get_state bitwise.  FB_E_INVAL for bad sizes or pointers, FB_E_NOMEM
 * for a short workspace. */
fb_status fb_hermite_steps_device(int32_t n_sys, int32_t n, const double *d_mass,
                                  double *d_pos, double *d_vel, int32_t *d_status,
                                  int64_t n_steps, double dt, void *d_workspace,
                                  size_t ws_bytes, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * fb_hermite_steps_device without a workspace.  The packed state lives in a
 * fixed 64 MiB array the library holds on each device it runs on until the
 * process ends (about 170000 three-body or 38000 sixteen-body systems);
 * larger batches fail with FB_E_NOMEM.  The call allocates nothing and
 * synchronises nothing.  Every call on one device shares that array: calls
 * whose work overlaps on one device (other streams, other threads) race and
 * must be serialised by the caller; work on one stream is ordered. */
fb_status fb_hermite_steps_device_noalloc(int32_t n_sys, int32_t n, const double *d_mass,
                                          double *d_pos, double *d_vel, int32_t *d_status,
                                          int64_t n_steps, double dt, void *hip_stream);

/* ---------------------------------------------------------------- plans */
/* The launch plan of body count n: lane mapping (FB_MAP_*) and waves per
 * workgroup (1..4) of its plain launches.  System-per-lane is built for
 * n <= 10 (n <= 8 with adaptive steps or stop rules); FB_MAP_AUTO (the
 * default) picks it for a bucket whose 64-system tiles give every SIMD of
 * the device a wavefront, and body-per-lane otherwise.  Entry n = 0 is the
 * fused persistent launch: its mapping selects the kernel class
 * (FB_MAP_SYSTEM_PER_LANE: full register file, system-per-lane tiles where n
 * allows; FB_MAP_BODY_PER_LANE: <= 128 VGPRs, body-per-lane tiles only;
 * FB_MAP_AUTO: the former when every bucket allows it and its tiles give
 * every SIMD a wavefront), plus waves per workgroup and workgroups per CU
 * (1..32, 0 = default).  In the system-per-lane class a body count whose own
 * plan is FB_MAP_BODY_PER_LANE runs body-per-lane tiles.  Plans are
 * process-wide; the autotuner sets them. */
fb_status fb_set_plan(int32_t n, int32_t mapping, int32_t waves_per_group,
                      int32_t groups_per_cu);
fb_status fb_get_plan(int32_t n, int32_t *mapping, int32_t *waves_per_group,
                      int32_t *groups_per_cu);

/* Autotuner (the counterpart of the paper's automatic choice of systems per
 * block under register/shared-memory/thread limits, Section 4.4, made by
 * measurement as its Section 5.3 recommends).  On ensemble e, for every body
 * count it holds, times `steps` fixed steps of dt with each candidate plan
 * of the plain schedule (mapping x waves per group), then the fused
 * persistent launch over the whole ensemble (waves per group x groups per
 * CU), and installs the fastest as the plans (fb_set_plan).  The ensemble's
 * state is restored afterwards.  out[0..max_out) receives every candidate
 * timed (n = 0 for the persistent launch); *n_out their count.  Allocates a
 * temporary copy of the ensemble's device state. */
typedef struct {
    int32_t n;                 /* body count; 0 = the persistent launch shape */
    int32_t mapping;           /* FB_MAP_*                                    */
    int32_t waves_per_group;
    int32_t groups_per_cu;
    double ms;                 /* elapsed time of the calibration run         */
    int32_t chosen;            /* 1 if installed as the plan                  */
    int32_t pad;
} fb_tune_entry;

fb_status fb_autotune(fb_ensemble *e, int64_t steps, double dt, fb_tune_entry *out,
                      int32_t max_out, int32_t *n_out);

/* ---------------------------------------------------------------- timing */
/* When enabled, the library brackets each integration kernel it launches
 * with HIP events on the ensemble's stream and accumulates their elapsed
 * time; fb_profile_read synchronises and returns (total ms, launches) since
 * the last reset. */
fb_status fb_profile_enable(int32_t on);
fb_status fb_profile_read(double *kernel_ms, int64_t *launches);

/* The device's achievable FP64 vector rate, for the roofline beside the
 * published peak: the best of two timed launches of independent FP64 FMA
 * chains (8 workgroups of 256 lanes per CU, 16 chains per lane), counted at
 * 2 flop per FMA, in TFLOP/s.  Allocates and frees its own buffers on the
 * current device and synchronises.  (A measurement utility; it computes
 * nothing of the method.) */
fb_status fb_fp64_fma_ceiling(double *tflops);

/* The device's LDS streaming rates per CU, in GB/s, for whole-wavefront
 * 16-byte reads (ds_read_b128) and writes (ds_write_b128): the best of two
 * timed launches (8 workgroups of 256 lanes per CU, each streaming 16 KB of
 * LDS slots, 64 consecutive per wavefront) per kind.  The body-per-lane
 * kernels exchange each evaluation's state through LDS (Section 4.2's
 * shared-memory staging), so these bound what an exchange costs.  Allocates
 * and frees its own buffers on the current device and synchronises.  (A
 * measurement utility; it computes nothing of the method.) */
fb_status fb_lds_rates(double *read_gbs_per_cu, double *write_gbs_per_cu);

/* The reciprocal square root every pair evaluation uses (Eq. 1's 1/|r|^3
 * and the jerk's 1/|r|^2 come from it; Section 4.4 discusses the hardware
 * rsqrt the paper relied on), applied elementwise to n DEVICE values x > 0:
 * d_out[i] = 1/sqrt(d_in[i]).  Asynchronous on the stream.  A measurement
 * utility for its accuracy; it computes nothing else. */
fb_status fb_eval_rsqrt(const double *d_in, double *d_out, int64_t n, void *hip_stream);

/* ---------------------------------------------------------------- serving */
/* A continuous-batching integration server.  Requests (an ensemble with its
 * own destination time and fixed step, integrated as fb_integrate does with
 * the persistent schedule) are queued from any thread and served by one
 * worker thread in quanta.  Queued requests are admitted in arrival order
 * while their device state fits the memory budget and the resident cap; a
 * request's systems take slots in server-wide pools, one per body count, so
 * the systems of many small requests fill the same tiles.  Each quantum
 * advances the scheduled requests' systems by up to steps_per_quantum steps
 * in one fused launch: every resident request (FB_POLICY_FAIR), or those
 * with at least long_steps steps left plus, least remaining work first,
 * others until they fill about quantum_tiles tiles (FB_POLICY_SRPT).
 * Finished requests are copied back and their memory is reused.  The kernel
 * mappings (the plan table's fused-kernel class in entry 0, auto meaning
 * body-per-lane, and per-n mappings) are fixed when the server is created,
 * so a request's results do not depend on what else is resident, on the
 * schedule or on later fb_set_plan calls.  (No counterpart in the paper,
 * whose host only sets up, loads, calls and examines -- Section 5.3; this is
 * the serving form of its many steps per kernel call.) */
typedef struct fb_server fb_server;

enum { FB_REQ_QUEUED = 0, FB_REQ_RUNNING = 1, FB_REQ_DONE = 2, FB_REQ_CANCELLED = 3,
       FB_REQ_FAILED = 4 };

enum { FB_POLICY_FAIR = 0, FB_POLICY_SRPT = 1 };

typedef struct {
    size_t budget_bytes;        /* device memory for resident requests, allocated
                                   once at creation (0: 4 GiB)                      */
    int32_t max_resident;       /* requests resident at once (0: 4096)              */
    int32_t steps_per_quantum;  /* steps per scheduled system per quantum (0: 2000) */
    int32_t policy;             /* FB_POLICY_FAIR / FB_POLICY_SRPT                  */
    int32_t quantum_tiles;      /* SRPT: tiles per quantum for the requests chosen
                                   by remaining work, whole requests (0: twice the
                                   waves the fused launch keeps resident)           */
    int32_t chunk_slots;        /* systems per pool chunk, multiple of 64 (0: 512)  */
    int32_t long_steps;         /* SRPT: requests with at least this many steps left
                                   run in every quantum, whatever their work, since
                                   their step count alone sets their latency (0: none) */
    int32_t idle_spread;        /* system-per-lane class: while a quantum's slowest
                                   tiles, not its total work, set its length, the
                                   slowest system-per-lane tiles run body-per-lane
                                   instead (a system over n lanes): shorter quanta
                                   under light load, bitwise the same results
                                   (0 or 1: on; -1: off)                            */
} fb_server_opts;

typedef struct {
    int64_t submitted, admitted, completed, queued, resident, quanta;
    double system_steps;        /* Hermite system-steps executed                    */
    double busy_seconds;        /* wall time spent inside quanta                    */
    size_t bytes_in_use, peak_bytes;
    int64_t spread_quanta;      /* quanta in which idle_spread moved system-per-lane
                                   tiles to body-per-lane                           */
} fb_server_stats;

void fb_server_opts_default(fb_server_opts *o);

/* Create a server on the current device.  hip_stream: the stream the worker
 * enqueues on (borrowed; NULL: the server creates its own).  Allocates the
 * whole budget up front; FB_E_NOMEM if that fails. */
fb_status fb_server_create(const fb_server_opts *o, void *hip_stream, fb_server **out);

/* Device bytes a request of these body counts needs on an empty server
 * with options o (NULL: defaults): its staging block plus whole pool chunks
 * for each body count.  0 on invalid input. */
size_t fb_server_request_bytes(const fb_server_opts *o, int32_t n_sys, const int32_t *n_body);

/* Queue a request; the host arrays are copied before the call returns
 * (layout as fb_ensemble_create, t0 = 0, 2..FB_MAX_SMALL_BODIES bodies per
 * system).  Integrates every system to t_end
 * with fixed step dt.  *req_id identifies it.  FB_E_INVAL on bad input,
 * FB_E_BUDGET if it would not fit the budget even on an empty server. */
fb_status fb_server_submit(fb_server *s, int32_t n_sys, const int32_t *n_body,
                           const double *mass, const double *pos, const double *vel,
                           double t_end, double dt, int64_t *req_id);

/* Current FB_REQ_* state of a request. */
fb_status fb_server_poll(fb_server *s, int64_t req_id, int32_t *state);

/* Block until the request is DONE, CANCELLED or FAILED, or timeout_s
 * seconds pass (< 0: no limit); *state (may be NULL) gets its state. */
fb_status fb_server_wait(fb_server *s, int64_t req_id, double timeout_s, int32_t *state);

/* Results of a DONE request into HOST arrays (any may be NULL; shapes as
 * fb_get_state), and times[3] = submit, admission and completion times on
 * the fb_monotonic_seconds clock.  Releases the request: a second call
 * returns FB_E_NOTFOUND.  FB_E_STATE if it is not done. */
fb_status fb_server_result(fb_server *s, int64_t req_id, double *pos, double *vel,
                           double *t, int32_t *status, int64_t *steps, double *times);

/* Cancel a queued or running request (it settles as CANCELLED). */
fb_status fb_server_cancel(fb_server *s, int64_t req_id);

/* Forget a settled (DONE, CANCELLED or FAILED) request without reading its
 * results, freeing what the server still holds for it; a later call on it
 * returns FB_E_NOTFOUND.  FB_E_STATE while it is queued or running. */
fb_status fb_server_release(fb_server *s, int64_t req_id);

fb_status fb_server_get_stats(fb_server *s, fb_server_stats *out);

/* Stop the worker (resident work is abandoned) and free the server. */
fb_status fb_server_destroy(fb_server *s);

/* Seconds on the host monotonic clock (CLOCK_MONOTONIC) used for times. */
double fb_monotonic_seconds(void);

/* ---------------------------------------------------------------- misc */
const char *fb_last_error(void);
const char *fb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FEWBODY_H */
