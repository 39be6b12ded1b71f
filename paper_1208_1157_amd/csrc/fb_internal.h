// Internal types shared by the HIP kernels (fb_kernels.hip) and the host
// runtime (fb_runtime.cpp).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fb {

// Rows of a bucket's structure-of-arrays state; row r, body b, slot s lives
// at st[(r * n + b) * pitch + s] (slot fastest: lanes read consecutive
// doubles).  a0/j0 are the carried acceleration and jerk of the step's last
// evaluation.
enum Row { R_M = 0, R_X = 1, R_V = 4, R_A = 7, R_J = 10, R_COUNT = 13 };

enum SysStatus {
    ST_ACTIVE = 0, ST_DONE = 1, ST_ENCOUNTER = 2, ST_EJECTED = 3,
    ST_NONFINITE = 4, ST_STALLED = 5, ST_MAXSTEPS = 6, ST_UNBOUND = 7
};

enum Mapping { MAP_SPL = 1, MAP_BPL = 2 };

constexpr int kMaxBodies = 16;         // kernels specialised per n exist for n <= 16
constexpr int kMaxLargeBodies = 512;   // larger systems run the runtime-n large-n kernels
constexpr int kMaxSplBodies = 10;      // plain system-per-lane instances exist for n <= 10
constexpr int kMaxSplAdv = 8;          // ... with adaptive steps / stop rules for n <= 8
constexpr int kMaxSplPersistent = 0;   // the body-per-lane fused class runs no system-per-lane tiles
constexpr int kMaxMvsBodies = 8;       // MVS kernels (system per lane) exist for n <= 8

// Device view of one homogeneous body-count bucket.  Per-slot arrays have
// `pitch` entries; slots [0, count) hold systems.
struct Bucket {
    double *st;          // [R_COUNT][n][pitch]
    double *t;           // current time
    double *t_end;       // destination time of the current run
    double *dt;          // fixed step of the current run
    double *dtn;         // carried adaptive step (<= 0: not yet proposed)
    double *t0run;       // time at the start of the current run
    long long *krun;     // whole steps taken in the current run
    long long *nfull;    // whole steps the current run takes before t_end
    long long *steps;    // steps since creation
    int *status;         // SysStatus
    int *orig;           // caller's index of the system in each slot
    int n, pitch, count, pad;
};

// One unit of persistent-schedule work: `count` systems of bucket `bucket`
// starting at `first` (a slot, or an index into an active list).
struct Tile {
    int bucket, first, count, kind;   // kind = mapping * 32 + n
};

struct StepParams {
    int adaptive;        // 0 fixed step, 1 adaptive step rule
    int stop_rules;      // bit 0 close encounter, bit 1 ejection
    double eta;
    double r_eject;
    long long max_steps; // per-system cap (LLONG_MAX: none)
    int quantum;         // at most this many steps per system per launch
    int pad;
};

// Compaction bookkeeping for the persistent schedule (device memory).
struct ActiveLists {
    int *cur;            // [sum pitch] active slots of each bucket, by bucket base
    int *next;           // survivors written by the running quantum
    int *base;           // [n_buckets] offset of each bucket's list
    int *cur_count;      // [n_buckets]
    int *next_count;     // [n_buckets]
};

inline int spl_tile_systems() { return 64; }
inline int bpl_tile_systems(int n) { return 64 / n; }
inline int tile_systems(int mapping, int n) {
    return mapping == MAP_SPL ? spl_tile_systems() : bpl_tile_systems(n);
}

// ---- launchers (fb_kernels.hip) -------------------------------------------
// pad_tail: also initialise slots count..pitch-1 as inert padding (a whole
// bucket); false for a view of a bucket shared with other owners.
hipError_t launch_pack(const Bucket &B, const double *mass, const double *pos,
                       const double *vel, const double *t0,
                       const long long *orig_off, int *bad, bool pad_tail, hipStream_t s);
hipError_t launch_prepare(const Bucket &B, hipStream_t s);
hipError_t launch_begin_run(const Bucket &B, int fixed_steps, long long n_steps,
                            double t_end, double dt, int adaptive, double eta,
                            hipStream_t s);
hipError_t launch_plain(const Bucket &B, int mapping, int waves_per_group,
                        const StepParams &P, hipStream_t s);
// spl_class: 0 = body-per-lane class fused kernel (<= 128 VGPRs; system-per-
// lane tiles for n <= kMaxSplPersistent), 1 = system-per-lane class (full
// register file; system-per-lane tiles for n <= kMaxSplBodies, or
// kMaxSplAdv with adaptive steps / stop rules).
hipError_t launch_persistent(const Bucket *d_buckets, const Tile *d_tiles,
                             const int *d_ntiles, int *d_head, const int *d_lists,
                             const StepParams &P, int adv, int spl_class, int grid,
                             int waves_per_group, ActiveLists *compact,
                             hipStream_t s);
hipError_t launch_build_tiles(const Bucket *d_buckets, int n_buckets,
                              const int *d_order, const int *d_mapping,
                              ActiveLists L, Tile *d_tiles, int *d_ntiles,
                              int *d_head, hipStream_t s);
hipError_t launch_reset_counter(int *p, int n, hipStream_t s);
hipError_t launch_unpack(const Bucket &B, const long long *orig_off, double *pos,
                         double *vel, double *acc, double *jerk, double *t,
                         int *status, long long *steps, double *dt_next,
                         hipStream_t s);
hipError_t launch_diag(const Bucket &B, double *energy, double *angmom, bool mvs_form,
                       hipStream_t s);
// Monitor record k of every system of B (kind 0 state, 1 star RV along the
// unit vector los, 2 energy and angular momentum) into a log buffer whose
// layout fb_log_bytes describes.
hipError_t launch_log(const Bucket &B, const long long *orig_off, int kind, const double *los,
                      int k, int max_records, double *out, hipStream_t s);
// Runge-Kutta Cash-Karp (body per lane, any n): fixed steps (eps == 0) or
// adaptive steps with error tolerance eps (P.adaptive nonzero).
hipError_t launch_plain_rkck(const Bucket &B, int waves_per_group, const StepParams &P,
                             double eps, hipStream_t s);
// Mixed-variable symplectic integrator (n <= kMaxMvsBodies, system per
// lane): conversion of a bucket to and from MVS form, fixed-step quanta, and
// read-back of a bucket in MVS form as inertial positions and velocities.
hipError_t launch_mvs_enter(const Bucket &B, hipStream_t s);
hipError_t launch_mvs_leave(const Bucket &B, hipStream_t s);
// mapping: MAP_SPL runs system per lane (n <= kMaxMvsBodies), MAP_BPL one
// body per lane across a workgroup (any n); the two give identical results.
hipError_t launch_plain_mvs(const Bucket &B, int mapping, int waves_per_group, const StepParams &P,
                            hipStream_t s);
hipError_t launch_unpack_mvs(const Bucket &B, const long long *orig_off, double *pos,
                             double *vel, double *t, int *status, long long *steps,
                             hipStream_t s);
hipError_t launch_count_active(const Bucket &B, int *count, hipStream_t s);
// Workgroup shape of the large-n kernels (n > kMaxBodies) with k bodies per
// lane: T lanes, a multiple of 64 up to 512 / k, holding S = floor(T / H)
// systems of H = ceil(n / k) lanes each; the T that leaves the fewest lanes
// idle.  S = 0 if the system does not fit.
void large_shape(int n, int k, int &T, int &S);
// Bodies per lane (1 or 2) of the large-n step kernel for n-body systems.
int large_bodies_per_lane(int n);
// FP64 FMA issue-ceiling probe: blocks x 256 lanes, iters x kFmaChains FMAs
// per lane (kFmaChains = 16); out holds blocks x 256 doubles.
hipError_t launch_fma_probe(double *out, int blocks, int iters, hipStream_t s);
// The pair evaluation's reciprocal square root, elementwise (accuracy check).
hipError_t launch_rsqrt(const double *in, double *out, long long n, hipStream_t s);
// Checkpoint restore of the carried (a0, j0), adaptive step, step count and
// status of every system of B from caller-order arrays.
hipError_t launch_restore(const Bucket &B, const long long *orig_off, const double *acc,
                          const double *jerk, const double *dtn, const long long *steps,
                          const int *status, hipStream_t s);
// Identity slot map and body offsets (o * n) of a single homogeneous bucket
// holding the caller's systems in order; clears *bad.
hipError_t launch_identity_tables(const Bucket &B, long long *orig_off, int *bad, hipStream_t s);
size_t persistent_lds_bytes(int spl_class, int waves_per_group);
int persistent_max_groups_per_cu(int adv, int spl_class, int waves_per_group);
// Largest n a persistent tile runs system-per-lane for, by kernel class.
inline int persistent_spl_limit(int spl_class, int adv)
{
    return spl_class ? (adv ? kMaxSplAdv : kMaxSplBodies) : kMaxSplPersistent;
}

}  // namespace fb
