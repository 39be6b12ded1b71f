// fb_runtime.cpp -- host runtime behind include/fewbody.h.
//
// An ensemble is laid out in device memory as one structure-of-arrays
// bucket per body count (systems of equal n side by side, slot fastest), so
// every launch is homogeneous in n and every load is coalesced.  The
// runtime owns the layout, the per-n launch plans, the plain (one launch per
// bucket) and persistent (one fused launch over a tile queue, optionally
// replayed as a captured HIP graph per quantum, with compaction of retired
// systems) schedules, and the HIP-event kernel timer.
#include "fewbody.h"
#include "fb_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fb_runtime_internal.h"

using namespace fb;
using namespace fb::rt;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
namespace {
// Message of the calling thread's last failure (a fixed buffer, so that
// reporting an error allocates nothing).
thread_local char g_err[512];
}  // namespace

namespace fb {
namespace rt {

fb_status fail(fb_status code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

fb_status hip_fail(hipError_t e, const char *what)
{
    return fail(e == hipErrorOutOfMemory ? FB_E_NOMEM : FB_E_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
namespace {
std::mutex g_plan_mu;
Plan g_plan[kMaxBodies + 1];
bool g_plan_init = false;

void init_plans_locked()
{
    if (g_plan_init)
        return;
    // Mapping chosen per bucket at launch (auto); four waves per group for
    // the register-light small systems, two otherwise.
    for (int n = 0; n <= kMaxBodies; ++n)
        g_plan[n] = Plan{0, n <= 3 ? 4 : 2, 0};
    g_plan[0] = Plan{0, 2, 8};   // fused-kernel class chosen per launch
    g_plan_init = true;
}
}  // namespace

Plan get_plan(int n)
{
    std::lock_guard<std::mutex> lk(g_plan_mu);
    init_plans_locked();
    Plan p = g_plan[n];
    if (n > 0 && p.mapping == MAP_SPL && n > kMaxSplBodies)
        p.mapping = MAP_BPL;
    return p;
}

// ---------------------------------------------------------------------------
// kernel timer (HIP events on the launch stream)
// ---------------------------------------------------------------------------
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_events;
double g_prof_ms = 0.0;
int64_t g_prof_launches = 0;

ProfScope::ProfScope(hipStream_t st) : s(st)
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        if (!g_prof_on)
            return;
        if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
            a = b = nullptr;
            return;
        }
        (void)hipEventRecord(a, s);
    }

ProfScope::~ProfScope()
    {
        if (!a)
            return;
        (void)hipEventRecord(b, s);
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_events.emplace_back(a, b);
    }

// ---------------------------------------------------------------------------
// layout
// ---------------------------------------------------------------------------
// Returns false for an invalid shape.
bool make_layout(int32_t n_sys, const int32_t *n_body, Layout &L)
{
    if (n_sys < 0 || (n_sys > 0 && !n_body))
        return false;
    std::vector<int> cnt(kMaxLargeBodies + 1, 0);
    int64_t nb = 0;
    for (int s = 0; s < n_sys; ++s) {
        if (n_body[s] < 2 || n_body[s] > kMaxLargeBodies)
            return false;
        cnt[n_body[s]]++;
        nb += n_body[s];
    }
    L.n_bodies = nb;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    L.max_tiles = 0;
    L.list_total = 0;
    for (int n = kMaxLargeBodies; n >= 2; --n) {   // buckets in descending n: longest work first
        if (!cnt[n])
            continue;
        BucketLayout bl;
        bl.n = n;
        bl.count = cnt[n];
        bl.pitch = (int)align_up((size_t)cnt[n], 64);
        const size_t P = bl.pitch;
        bl.st = take(sizeof(double) * R_COUNT * n * P);
        bl.t = take(8 * P);
        bl.t_end = take(8 * P);
        bl.dt = take(8 * P);
        bl.dtn = take(8 * P);
        bl.t0run = take(8 * P);
        bl.krun = take(8 * P);
        bl.nfull = take(8 * P);
        bl.steps = take(8 * P);
        bl.status = take(4 * P);
        bl.orig = take(4 * P);
        const int per_tile = std::max(1, 64 / n);
        L.max_tiles += (cnt[n] + per_tile - 1) / per_tile;
        L.list_total += bl.pitch;
        L.b.push_back(bl);
    }
    const size_t nbk = L.b.size();
    L.buckets = take(sizeof(Bucket) * std::max<size_t>(nbk, 1));
    L.orig_off = take(8 * ((size_t)n_sys + 1));
    L.staging = take(8 * (12 * (size_t)nb + 4 * (size_t)n_sys + 1));
    L.diag = take(8 * 4 * ((size_t)n_sys + 1));
    L.ints = take(4 * 64);
    L.tiles = take(sizeof(Tile) * ((size_t)L.max_tiles + 1));
    L.lists0 = take(4 * ((size_t)L.list_total + 1));
    L.lists1 = take(4 * ((size_t)L.list_total + 1));
    L.list_base = take(4 * (nbk + 1));
    L.counts0 = take(4 * (nbk + 1));
    L.counts1 = take(4 * (nbk + 1));
    L.order = take(4 * (nbk + 1));
    L.mapping = take(4 * (nbk + 1));
    L.total = off;
    return true;
}

std::vector<Bucket> bucket_views(char *base, const Layout &L)
{
    std::vector<Bucket> out;
    for (const BucketLayout &bl : L.b) {
        Bucket B;
        B.st = reinterpret_cast<double *>(base + bl.st);
        B.t = reinterpret_cast<double *>(base + bl.t);
        B.t_end = reinterpret_cast<double *>(base + bl.t_end);
        B.dt = reinterpret_cast<double *>(base + bl.dt);
        B.dtn = reinterpret_cast<double *>(base + bl.dtn);
        B.t0run = reinterpret_cast<double *>(base + bl.t0run);
        B.krun = reinterpret_cast<long long *>(base + bl.krun);
        B.nfull = reinterpret_cast<long long *>(base + bl.nfull);
        B.steps = reinterpret_cast<long long *>(base + bl.steps);
        B.status = reinterpret_cast<int *>(base + bl.status);
        B.orig = reinterpret_cast<int *>(base + bl.orig);
        B.n = bl.n;
        B.pitch = bl.pitch;
        B.count = bl.count;
        B.pad = 0;
        out.push_back(B);
    }
    return out;
}

std::vector<int> slot_origins(const std::vector<int32_t> &n_body, const Bucket &B)
{
    std::vector<int> v;
    v.reserve(B.pitch);
    for (size_t s = 0; s < n_body.size(); ++s)
        if (n_body[s] == B.n)
            v.push_back((int)s);
    v.resize(B.pitch, 0);
    return v;
}

}  // namespace rt
}  // namespace fb

// ---------------------------------------------------------------------------
// ensemble object
// ---------------------------------------------------------------------------
struct fb_ensemble {
    int device = 0;
    int num_cu = 256;
    hipStream_t stream = nullptr;
    int32_t n_sys = 0;
    std::vector<int32_t> n_body;
    Layout L;
    char *base = nullptr;
    bool owns = false;
    std::vector<Bucket> buckets;    // host copies of the device views
    Bucket *d_buckets = nullptr;
    long long *d_orig_off = nullptr;
    double *d_staging = nullptr;
    double *d_diag = nullptr;
    int *d_ints = nullptr;          // [0] bad flag, [1] ntiles, [2] head, [3] active count
    Tile *d_tiles = nullptr;
    int *d_lists[2] = {nullptr, nullptr};
    int *d_list_base = nullptr;
    int *d_counts[2] = {nullptr, nullptr};
    int *d_order = nullptr;
    int *d_mapping = nullptr;
    int *h_pinned = nullptr;        // pinned host ints for control reads
    hipStream_t capture_stream = nullptr;
    // What the state rows hold: (x, v, a0, j0) ready for Hermite; the MVS
    // variables; or (x, v) with (a0, j0) stale after a Runge-Kutta run.
    enum Form { FORM_HERMITE, FORM_MVS, FORM_XV } form = FORM_HERMITE;
    bool mvs_form() const { return form == FORM_MVS; }
};

namespace {

template <class T>
T *at(fb_ensemble *e, size_t off)
{
    return reinterpret_cast<T *>(e->base + off);
}

fb_status bind_layout(fb_ensemble *e)
{
    e->buckets = bucket_views(e->base, e->L);
    e->d_buckets = at<Bucket>(e, e->L.buckets);
    e->d_orig_off = at<long long>(e, e->L.orig_off);
    e->d_staging = at<double>(e, e->L.staging);
    e->d_diag = at<double>(e, e->L.diag);
    e->d_ints = at<int>(e, e->L.ints);
    e->d_tiles = at<Tile>(e, e->L.tiles);
    e->d_lists[0] = at<int>(e, e->L.lists0);
    e->d_lists[1] = at<int>(e, e->L.lists1);
    e->d_list_base = at<int>(e, e->L.list_base);
    e->d_counts[0] = at<int>(e, e->L.counts0);
    e->d_counts[1] = at<int>(e, e->L.counts1);
    e->d_order = at<int>(e, e->L.order);
    e->d_mapping = at<int>(e, e->L.mapping);
    return FB_OK;
}

// Upload the host-side tables (bucket views, slot -> caller index map, body
// offsets, list bases) with synchronous copies; the staging of the inputs
// must already be enqueued or resident.
fb_status upload_tables(fb_ensemble *e)
{
    const int ns = e->n_sys;
    std::vector<long long> off(ns + 1, 0);
    for (int s = 0; s < ns; ++s)
        off[s + 1] = off[s] + e->n_body[s];
    FB_HIP(hipMemcpyAsync(e->d_orig_off, off.data(), sizeof(long long) * (ns + 1),
                          hipMemcpyHostToDevice, e->stream));
    std::vector<int> list_base;
    int acc = 0;
    std::vector<std::vector<int>> origins;
    for (const Bucket &B : e->buckets) {
        origins.push_back(slot_origins(e->n_body, B));
        FB_HIP(hipMemcpyAsync(B.orig, origins.back().data(), sizeof(int) * B.pitch,
                              hipMemcpyHostToDevice, e->stream));
        list_base.push_back(acc);
        acc += B.pitch;
    }
    const int nbk = (int)e->buckets.size();
    if (nbk) {
        FB_HIP(hipMemcpyAsync(e->d_buckets, e->buckets.data(), sizeof(Bucket) * nbk,
                              hipMemcpyHostToDevice, e->stream));
        FB_HIP(hipMemcpyAsync(e->d_list_base, list_base.data(), sizeof(int) * nbk,
                              hipMemcpyHostToDevice, e->stream));
        std::vector<int> order(nbk);
        for (int i = 0; i < nbk; ++i)
            order[i] = i;   // buckets are laid out in descending n already
        FB_HIP(hipMemcpyAsync(e->d_order, order.data(), sizeof(int) * nbk, hipMemcpyHostToDevice,
                              e->stream));
    }
    // the vectors above die at return: wait for the copies
    FB_HIP(hipStreamSynchronize(e->stream));
    return FB_OK;
}

fb_status finish_create(fb_ensemble *e, const double *d_mass, const double *d_pos,
                        const double *d_vel, const double *d_t0)
{
    fb_status st = upload_tables(e);
    if (st != FB_OK)
        return st;
    FB_HIP(launch_reset_counter(e->d_ints, 64, e->stream));
    for (const Bucket &B : e->buckets)
        FB_HIP(launch_pack(B, d_mass, d_pos, d_vel, d_t0, e->d_orig_off, e->d_ints, true, e->stream));
    for (const Bucket &B : e->buckets)
        FB_HIP(launch_prepare(B, e->stream));
    FB_HIP(hipMemcpyAsync(e->h_pinned, e->d_ints, sizeof(int), hipMemcpyDeviceToHost, e->stream));
    FB_HIP(hipStreamSynchronize(e->stream));
    if (e->h_pinned[0])
        return fail(FB_E_INVAL, "mass must be finite and >= 0; pos, vel and t0 finite");
    return FB_OK;
}

fb_status alloc_common(fb_ensemble *e, void *hip_stream)
{
    e->stream = (hipStream_t)hip_stream;
    FB_HIP(hipGetDevice(&e->device));
    hipDeviceProp_t prop;
    FB_HIP(hipGetDeviceProperties(&prop, e->device));
    e->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    FB_HIP(hipHostMalloc((void **)&e->h_pinned, 64 * sizeof(int), hipHostMallocDefault));
    return FB_OK;
}

void free_ensemble(fb_ensemble *e)
{
    if (!e)
        return;
    if (e->owns && e->base)
        (void)hipFree(e->base);
    if (e->h_pinned)
        (void)hipHostFree(e->h_pinned);
    if (e->capture_stream)
        (void)hipStreamDestroy(e->capture_stream);
    delete e;
}

bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i]))
            return false;
    return true;
}

StepParams make_params(const fb_opts &o, int quantum)
{
    StepParams P;
    P.adaptive = o.adaptive == 2 ? 2 : (o.adaptive ? 1 : 0);
    P.stop_rules = o.stop_rules & (FB_STOP_ENCOUNTER | FB_STOP_EJECT);
    P.eta = o.eta;
    P.r_eject = o.r_eject;
    P.max_steps = o.max_steps > 0 ? (long long)o.max_steps : LLONG_MAX;
    P.quantum = quantum;
    P.pad = 0;
    return P;
}

fb_status check_opts(const fb_opts &o)
{
    if (o.adaptive < 0 || o.adaptive > 2)
        return fail(FB_E_INVAL, "adaptive must be 0 (fixed), 1 (pairwise rule) or 2 (Eq. 5 rule)");
    if (o.adaptive && !(std::isfinite(o.eta) && o.eta > 0.0))
        return fail(FB_E_INVAL, "eta must be finite and > 0");
    if ((o.stop_rules & FB_STOP_EJECT) && !(o.r_eject > 0.0))
        return fail(FB_E_INVAL, "r_eject must be > 0");
    if (o.schedule != FB_SCHED_PLAIN && o.schedule != FB_SCHED_PERSISTENT)
        return fail(FB_E_INVAL, "unknown schedule %d", o.schedule);
    return FB_OK;
}

// Number of systems still ACTIVE (synchronises the stream).
fb_status count_active(fb_ensemble *e, int &out)
{
    FB_HIP(launch_reset_counter(e->d_ints + 3, 1, e->stream));
    for (const Bucket &B : e->buckets)
        FB_HIP(launch_count_active(B, e->d_ints + 3, e->stream));
    FB_HIP(hipMemcpyAsync(e->h_pinned + 3, e->d_ints + 3, sizeof(int), hipMemcpyDeviceToHost,
                          e->stream));
    FB_HIP(hipStreamSynchronize(e->stream));
    out = e->h_pinned[3];
    return FB_OK;
}

// Waves per SIMD below which the survivors of a compacted persistent run
// (automatic class) move to the full-register kernel class with body-per-
// lane tiles and unrolled partner loops: one wave per SIMD, more work in
// flight per wave.
#ifndef FB_TAIL_WAVES_PER_SIMD
#define FB_TAIL_WAVES_PER_SIMD 2
#endif

// Plain schedule: one launch per bucket (one per quantum if quanta are set).
fb_status run_plain(fb_ensemble *e, const fb_opts &o, long long step_bound)
{
    const int quantum = o.steps_per_quantum > 0 ? o.steps_per_quantum : INT_MAX;
    for (;;) {
        for (const Bucket &B : e->buckets) {
            const Plan p = B.n <= kMaxBodies ? get_plan(B.n) : Plan{MAP_BPL, 1, 0};
            const StepParams P = make_params(o, quantum);
            const int map = plain_mapping(p, B, P.adaptive || P.stop_rules, e->num_cu);
            ProfScope ps(e->stream);
            FB_HIP(launch_plain(B, map, p.waves_per_group, P, e->stream));
        }
        if (quantum == INT_MAX)
            return FB_OK;
        if (step_bound >= 0) {
            step_bound -= quantum;
            if (step_bound <= 0)
                return FB_OK;
            continue;
        }
        int act = 0;
        fb_status st = count_active(e, act);
        if (st != FB_OK)
            return st;
        if (act == 0)
            return FB_OK;
    }
}

// Persistent schedule: one fused launch per quantum over a tile queue; the
// tiles cover every bucket, largest n first.  With compaction the tiles of
// each quantum are rebuilt on the device from the previous quantum's
// survivors.  Quanta are captured once into a HIP graph (two quanta, so the
// survivor lists alternate) and replayed.
fb_status run_persistent(fb_ensemble *e, const fb_opts &o, long long step_bound)
{
    const int nbk = (int)e->buckets.size();
    if (nbk == 0)
        return FB_OK;
    // Buckets are laid out in descending n: the large-n ones (n > kMaxBodies)
    // come first and run their own plain launches inside every quantum; the
    // fused launch's tile queue covers the others.
    int n_large = 0;
    while (n_large < nbk && e->buckets[n_large].n > kMaxBodies)
        ++n_large;
    const int nb_small = nbk - n_large;
    const std::vector<Bucket> small(e->buckets.begin() + n_large, e->buckets.end());
    const Plan p0 = get_plan(0);
    const int W = std::max(1, std::min(4, p0.waves_per_group));
    const bool adv = o.adaptive || o.stop_rules;
    const int quantum = o.steps_per_quantum > 0 ? o.steps_per_quantum : INT_MAX;
    StepParams P = make_params(o, quantum);
    const bool compact = o.compact != 0;
    int cls = persistent_class(p0, small, adv, e->num_cu);

    // Lists (identity) and counts of every bucket; mapping and tile order of
    // the small buckets.
    std::vector<int> counts(nbk, 0), order, ident;
    for (int i = n_large; i < nbk; ++i) {
        order.push_back(i);
        counts[i] = e->buckets[i].count;
    }
    ident.reserve(e->L.list_total);
    for (const Bucket &B : e->buckets)
        for (int s = 0; s < B.pitch; ++s)
            ident.push_back(s);
    if (nb_small)
        FB_HIP(hipMemcpyAsync(e->d_order, order.data(), sizeof(int) * nb_small,
                              hipMemcpyHostToDevice, e->stream));
    FB_HIP(hipMemcpyAsync(e->d_lists[0], ident.data(), sizeof(int) * ident.size(),
                          hipMemcpyHostToDevice, e->stream));
    FB_HIP(hipMemcpyAsync(e->d_counts[0], counts.data(), sizeof(int) * nbk, hipMemcpyHostToDevice,
                          e->stream));
    std::vector<int> mapping(nbk, MAP_BPL);
    int grid = 1;
    // Per-bucket mappings and grid of fused-kernel class c; all_bpl runs
    // every tile body-per-lane (in the system-per-lane class: one wave per
    // SIMD with the full register file, partner loops unrolled).
    auto set_class = [&](int c, bool all_bpl) -> hipError_t {
        const int spl_lim = all_bpl ? 0 : persistent_spl_limit(c, adv ? 1 : 0);
        for (int i = n_large; i < nbk; ++i) {
            const int n = e->buckets[i].n;
            const int m = get_plan(n).mapping;
            // in the system-per-lane class every bucket that can runs system-
            // per-lane, unless its plan asks for body-per-lane
            mapping[i] = (n <= spl_lim && m != MAP_BPL && (m == MAP_SPL || c == 1)) ? MAP_SPL
                                                                                   : MAP_BPL;
        }
        int gpc = p0.groups_per_cu > 0 ? p0.groups_per_cu : 8;
        const int occ = persistent_max_groups_per_cu(adv ? 1 : 0, c, W);
        if (occ > 0)
            gpc = std::min(gpc, occ);
        grid = std::max(1, gpc * e->num_cu);
        cls = c;
        hipError_t err = hipMemcpyAsync(e->d_mapping, mapping.data(), sizeof(int) * nbk,
                                        hipMemcpyHostToDevice, e->stream);
        if (err == hipSuccess)   // the host vector is rewritten by the next switch
            err = hipStreamSynchronize(e->stream);
        return err;
    };
    FB_HIP(set_class(cls, false));   // also waits for the copies above (host vectors die at return)
    bool tail_mode = false;

    ActiveLists AL[2];
    for (int k = 0; k < 2; ++k) {
        AL[k].cur = e->d_lists[k];
        AL[k].next = e->d_lists[1 - k];
        AL[k].base = e->d_list_base;
        AL[k].cur_count = e->d_counts[k];
        AL[k].next_count = e->d_counts[1 - k];
    }
    int *d_ntiles = e->d_ints + 1, *d_head = e->d_ints + 2;

    // Enqueue one quantum.  With compaction it reads lists/counts [k] and
    // writes the survivors to [1-k]; without, every quantum re-runs the
    // identity lists [0] (retired systems exit at once).
    auto quantum_launch = [&](hipStream_t s, int k) -> hipError_t {
        if (!compact)
            k = 0;
        for (int i = 0; i < n_large; ++i) {
            const hipError_t err = launch_plain(e->buckets[i], MAP_BPL, 1, P, s);
            if (err != hipSuccess)
                return err;
        }
        if (nb_small == 0)
            return hipSuccess;
        hipError_t err = launch_build_tiles(e->d_buckets, nb_small, e->d_order, e->d_mapping,
                                            AL[k], e->d_tiles, d_ntiles, d_head, s);
        if (err != hipSuccess)
            return err;
        ActiveLists al = AL[k];
        return launch_persistent(e->d_buckets, e->d_tiles, d_ntiles, d_head, e->d_lists[k], P,
                                 adv ? 1 : 0, cls, grid, W, compact ? &al : nullptr, s);
    };

    if (quantum == INT_MAX) {
        ProfScope ps(e->stream);
        FB_HIP(quantum_launch(e->stream, 0));
        return FB_OK;
    }

    // capture two quanta (0 -> 1 -> 0) into a graph
    if (!e->capture_stream)
        FB_HIP(hipStreamCreateWithFlags(&e->capture_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto release = [&]() {
        if (exec)
            (void)hipGraphExecDestroy(exec);
        if (graph)
            (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    };
    auto capture = [&]() -> fb_status {
        release();
        FB_HIP(hipStreamBeginCapture(e->capture_stream, hipStreamCaptureModeThreadLocal));
        hipError_t cerr = quantum_launch(e->capture_stream, 0);
        if (cerr == hipSuccess)
            cerr = quantum_launch(e->capture_stream, 1);
        hipError_t eerr = hipStreamEndCapture(e->capture_stream, &graph);
        if (cerr != hipSuccess)
            return hip_fail(cerr, "quantum capture");
        FB_HIP(eerr);
        hipError_t ierr = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (ierr != hipSuccess)
            return hip_fail(ierr, "hipGraphInstantiate");
        return FB_OK;
    };
    fb_status result = capture();
    long long done_steps = 0;
    while (result == FB_OK) {
        {
            ProfScope ps(e->stream);
            hipError_t err = hipGraphLaunch(exec, e->stream);
            if (err != hipSuccess) {
                result = hip_fail(err, "hipGraphLaunch");
                break;
            }
        }
        done_steps += 2LL * quantum;
        if (step_bound >= 0) {
            if (done_steps >= step_bound)
                break;
            continue;
        }
        long long act = 0, spl_tiles = 0, bpl_waves = 0;
        if (compact) {
            // survivors of the second quantum sit in counts[0] (the small
            // buckets' entries; at most kMaxBodies - 1 of them)
            hipError_t err = hipSuccess;
            if (nb_small)
                err = hipMemcpyAsync(e->h_pinned + 8, e->d_counts[0] + n_large,
                                     sizeof(int) * nb_small, hipMemcpyDeviceToHost, e->stream);
            if (err == hipSuccess)
                err = hipStreamSynchronize(e->stream);
            if (err != hipSuccess) {
                result = hip_fail(err, "active count");
                break;
            }
            for (int i = 0; i < nb_small; ++i) {
                const int c = e->h_pinned[8 + i], per = 64 / e->buckets[n_large + i].n;
                act += c;
                spl_tiles += (c + 63) / 64;
                bpl_waves += (c + per - 1) / per;
            }
            if (n_large) {   // the large buckets keep no survivor lists
                FB_HIP(launch_reset_counter(e->d_ints + 3, 1, e->stream));
                for (int i = 0; i < n_large; ++i)
                    FB_HIP(launch_count_active(e->buckets[i], e->d_ints + 3, e->stream));
                FB_HIP(hipMemcpyAsync(e->h_pinned + 3, e->d_ints + 3, sizeof(int),
                                      hipMemcpyDeviceToHost, e->stream));
                FB_HIP(hipStreamSynchronize(e->stream));
                act += e->h_pinned[3];
            }
        } else {
            int a = 0;
            result = count_active(e, a);
            if (result != FB_OK)
                break;
            act = a;
        }
        if (act == 0)
            break;
        // As survivors thin out (automatic class only): the system-per-lane
        // class runs one wavefront per SIMD, so once the survivors' 64-system
        // tiles no longer give every SIMD one, the body-per-lane class (a
        // system over n lanes) keeps more of the device busy; once even its
        // waves no longer give every SIMD two, each wave may as well have
        // its SIMD's whole register file, and the full-register kernel runs
        // the body-per-lane tiles with their partner loops unrolled (more
        // independent work in flight per wave).  All these compute bitwise
        // the same states, so the switches are invisible in the results.
        bool recapture = false;
        if (compact && p0.mapping == 0 && !tail_mode) {
            int to = -1;
            bool all_bpl = false;
            if (bpl_waves < (long long)FB_TAIL_WAVES_PER_SIMD * 4 * e->num_cu) {
                to = 1;
                all_bpl = true;
            } else if (cls == 1 && spl_tiles < 4LL * e->num_cu) {
                to = 0;
            }
            if (to >= 0) {
                hipError_t err = set_class(to, all_bpl);
                if (err != hipSuccess) {
                    result = hip_fail(err, "class switch");
                    break;
                }
                tail_mode = all_bpl;
                recapture = true;
            }
        }
        // Once every surviving tile has a wave of its own, compaction has
        // nothing left to gain and a quantum boundary only makes each tile
        // wait for the slowest one (8-body tiles take about 1.7x as long per
        // step as 4-body ones, and the tiles' step counts differ), so the
        // tiles run on to their ends in one launch.
        if (tail_mode && P.quantum == quantum && bpl_waves <= (long long)grid * W) {
            P.quantum = INT_MAX / 2;
            recapture = true;
        }
        if (recapture)
            result = capture();
    }
    release();
    return result;
}

// Back from MVS form to the Hermite state: inertial (x, v) and a fresh
// set-up evaluation of (a0, j0).
fb_status ensure_inertial(fb_ensemble *e)
{
    if (e->form == fb_ensemble::FORM_HERMITE)
        return FB_OK;
    for (const Bucket &B : e->buckets) {
        if (e->form == fb_ensemble::FORM_MVS)
            FB_HIP(launch_mvs_leave(B, e->stream));
        FB_HIP(launch_prepare(B, e->stream));
    }
    e->form = fb_ensemble::FORM_HERMITE;
    return FB_OK;
}

// (x, v) in the rows, for integrators that carry nothing else.
fb_status ensure_xv(fb_ensemble *e)
{
    if (e->form == fb_ensemble::FORM_MVS) {
        for (const Bucket &B : e->buckets)
            FB_HIP(launch_mvs_leave(B, e->stream));
        e->form = fb_ensemble::FORM_XV;
    }
    return FB_OK;
}

// Runge-Kutta quanta: one body-per-lane launch per bucket and quantum.
fb_status run_rkck(fb_ensemble *e, const fb_opts &o, int adaptive, double eps,
                   long long step_bound)
{
    const int quantum = o.steps_per_quantum > 0 ? o.steps_per_quantum : INT_MAX;
    for (;;) {
        for (const Bucket &B : e->buckets) {
            StepParams P = make_params(o, quantum);
            P.adaptive = adaptive;
            ProfScope ps(e->stream);
            FB_HIP(launch_plain_rkck(B, 2, P, eps, e->stream));
        }
        if (quantum == INT_MAX)
            return FB_OK;
        if (step_bound >= 0) {
            step_bound -= quantum;
            if (step_bound <= 0)
                return FB_OK;
            continue;
        }
        int act = 0;
        fb_status st = count_active(e, act);
        if (st != FB_OK)
            return st;
        if (act == 0)
            return FB_OK;
    }
}

bool has_large(const fb_ensemble *e)
{
    for (const Bucket &B : e->buckets)
        if (B.n > kMaxBodies)
            return true;
    return false;
}

// Systems of more than kMaxBodies bodies run the large-n kernels (on the
// persistent schedule as plain launches inside every quantum); nothing is
// refused for them today.
fb_status check_large(const fb_ensemble *, const fb_opts &)
{
    return FB_OK;
}

fb_status check_rk_opts(const fb_opts &o)
{
    if (o.adaptive || o.stop_rules || o.compact || o.schedule != FB_SCHED_PLAIN)
        return fail(FB_E_INVAL, "Runge-Kutta takes the plain schedule without stop rules "
                                "(opts.adaptive, stop_rules and compact must be 0, schedule plain)");
    return check_opts(o);
}

// MVS quanta: one system-per-lane launch per bucket and quantum.
fb_status run_mvs(fb_ensemble *e, const fb_opts &o, long long step_bound)
{
    const int quantum = o.steps_per_quantum > 0 ? o.steps_per_quantum : INT_MAX;
    for (;;) {
        for (const Bucket &B : e->buckets) {
            const StepParams P = make_params(o, quantum);
            ProfScope ps(e->stream);
            // the Hermite plan's mapping rule (system per lane when its
            // 64-system tiles fill the device), within MVS's own limit
            const Plan p = B.n <= kMaxBodies ? get_plan(B.n) : Plan{MAP_BPL, 1, 0};
            const int map = B.n > kMaxMvsBodies ? MAP_BPL : plain_mapping(p, B, false, e->num_cu);
            FB_HIP(launch_plain_mvs(B, map, 1, P, e->stream));
        }
        if (quantum == INT_MAX)
            return FB_OK;
        step_bound -= quantum;
        if (step_bound <= 0)
            return FB_OK;
    }
}

// A log spec for a run that writes `records` records: kind, capacity, buffer
// size and (FB_LOG_RV) the line of sight, returned normalised in los.
fb_status check_log(const fb_ensemble *e, const fb_log_spec *log, long long records,
                    double (&los)[3])
{
    if (log->max_records < 1)
        return fail(FB_E_INVAL, "log.max_records must be >= 1");
    if (records > log->max_records)
        return fail(FB_E_INVAL, "the run makes %lld records, log.max_records is %d", records,
                    log->max_records);
    if (log->kind != FB_LOG_STATE && log->kind != FB_LOG_RV && log->kind != FB_LOG_ENERGY)
        return fail(FB_E_INVAL, "unknown log kind %d", log->kind);
    const size_t need = fb_log_bytes(e->n_sys, e->n_body.data(), log->kind, log->max_records);
    if (e->n_sys > 0 && (!log->d_buffer || log->buffer_bytes < need))
        return fail(FB_E_INVAL, "log buffer of %zu bytes, %zu needed", log->buffer_bytes, need);
    los[0] = 0.0;
    los[1] = 0.0;
    los[2] = 1.0;
    if (log->kind == FB_LOG_RV) {
        const double l2 = log->los[0] * log->los[0] + log->los[1] * log->los[1] +
                          log->los[2] * log->los[2];
        if (!(std::isfinite(l2) && l2 > 0.0))
            return fail(FB_E_INVAL, "log.los must be a finite non-zero vector");
        const double inv = 1.0 / std::sqrt(l2);
        for (int c = 0; c < 3; ++c)
            los[c] = log->los[c] * inv;
    }
    return FB_OK;
}

fb_status run(fb_ensemble *e, const fb_opts &o, long long step_bound)
{
    if (o.schedule == FB_SCHED_PERSISTENT)
        return run_persistent(e, o, step_bound);
    return run_plain(e, o, step_bound);
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

void fb_opts_default(fb_opts *o)
{
    if (!o)
        return;
    std::memset(o, 0, sizeof *o);
    o->adaptive = 0;
    o->eta = 0.01;
    o->stop_rules = 0;
    o->r_eject = 100.0;
    o->max_steps = 0;
    o->schedule = FB_SCHED_PLAIN;
    o->steps_per_quantum = 0;
    o->compact = 0;
}

size_t fb_workspace_bytes(int32_t n_sys, const int32_t *n_body)
{
    Layout L;
    if (!make_layout(n_sys, n_body, L))
        return 0;
    return L.total;
}

fb_status fb_ensemble_create(int32_t n_sys, const int32_t *n_body, const double *mass,
                             const double *pos, const double *vel, const double *t0,
                             void *hip_stream, fb_ensemble **out)
{
    if (!out)
        return fail(FB_E_INVAL, "out is NULL");
    *out = nullptr;
    Layout L;
    if (!make_layout(n_sys, n_body, L))
        return fail(FB_E_INVAL, "n_sys must be >= 0 and every n_body in 2..%d", kMaxLargeBodies);
    const size_t N = (size_t)L.n_bodies;
    if (N && (!mass || !pos || !vel))
        return fail(FB_E_INVAL, "mass, pos and vel are required");
    for (size_t i = 0; i < N; ++i)
        if (!(std::isfinite(mass[i]) && mass[i] >= 0.0))
            return fail(FB_E_INVAL, "mass[%zu] must be finite and >= 0", i);
    if (!finite_all(pos, 3 * N) || !finite_all(vel, 3 * N))
        return fail(FB_E_INVAL, "pos and vel must be finite");
    if (t0 && !finite_all(t0, (size_t)n_sys))
        return fail(FB_E_INVAL, "t0 must be finite");
    fb_ensemble *e = new fb_ensemble();
    e->n_sys = n_sys;
    e->n_body.assign(n_body, n_body + n_sys);
    e->L = L;
    fb_status st = alloc_common(e, hip_stream);
    if (st != FB_OK) {
        free_ensemble(e);
        return st;
    }
    hipError_t err = hipMalloc((void **)&e->base, L.total);
    if (err != hipSuccess) {
        free_ensemble(e);
        return hip_fail(err, "hipMalloc(ensemble)");
    }
    e->owns = true;
    bind_layout(e);
    // stage the inputs: mass | pos | vel | t0
    double *d_mass = e->d_staging, *d_pos = d_mass + N, *d_vel = d_pos + 3 * N;
    double *d_t0 = t0 ? d_vel + 3 * N : nullptr;
    err = hipMemcpyAsync(d_mass, mass, 8 * N, hipMemcpyHostToDevice, e->stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(d_pos, pos, 24 * N, hipMemcpyHostToDevice, e->stream);
    if (err == hipSuccess)
        err = hipMemcpyAsync(d_vel, vel, 24 * N, hipMemcpyHostToDevice, e->stream);
    if (err == hipSuccess && t0)
        err = hipMemcpyAsync(d_t0, t0, 8 * (size_t)n_sys, hipMemcpyHostToDevice, e->stream);
    if (err != hipSuccess) {
        free_ensemble(e);
        return hip_fail(err, "input upload");
    }
    st = finish_create(e, d_mass, d_pos, d_vel, d_t0);
    if (st != FB_OK) {
        free_ensemble(e);
        return st;
    }
    *out = e;
    return FB_OK;
}

fb_status fb_ensemble_create_device(int32_t n_sys, const int32_t *n_body, const double *d_mass,
                                    const double *d_pos, const double *d_vel, const double *d_t0,
                                    void *d_workspace, size_t ws_bytes, void *hip_stream,
                                    fb_ensemble **out)
{
    if (!out)
        return fail(FB_E_INVAL, "out is NULL");
    *out = nullptr;
    Layout L;
    if (!make_layout(n_sys, n_body, L))
        return fail(FB_E_INVAL, "n_sys must be >= 0 and every n_body in 2..%d", kMaxLargeBodies);
    if (L.n_bodies && (!d_mass || !d_pos || !d_vel))
        return fail(FB_E_INVAL, "d_mass, d_pos and d_vel are required");
    if (!d_workspace || ws_bytes < L.total)
        return fail(FB_E_NOMEM, "workspace of %zu bytes needed, %zu given", L.total, ws_bytes);
    if (((uintptr_t)d_workspace) % 256)
        return fail(FB_E_INVAL, "workspace must be 256-byte aligned");
    fb_ensemble *e = new fb_ensemble();
    e->n_sys = n_sys;
    e->n_body.assign(n_body, n_body + n_sys);
    e->L = L;
    fb_status st = alloc_common(e, hip_stream);
    if (st != FB_OK) {
        free_ensemble(e);
        return st;
    }
    e->base = (char *)d_workspace;
    e->owns = false;
    bind_layout(e);
    st = finish_create(e, d_mass, d_pos, d_vel, d_t0);
    if (st != FB_OK) {
        free_ensemble(e);
        return st;
    }
    *out = e;
    return FB_OK;
}

fb_status fb_ensemble_restore(int32_t n_sys, const int32_t *n_body, const double *mass,
                              const double *pos, const double *vel, const double *acc0,
                              const double *jerk0, const double *t, const double *dt_next,
                              const int32_t *status, const int64_t *steps, void *hip_stream,
                              fb_ensemble **out)
{
    if (!out)
        return fail(FB_E_INVAL, "out is NULL");
    *out = nullptr;
    Layout L;
    if (!make_layout(n_sys, n_body, L))
        return fail(FB_E_INVAL, "n_sys must be >= 0 and every n_body in 2..%d", kMaxLargeBodies);
    const size_t N = (size_t)L.n_bodies, ns = (size_t)n_sys;
    if (N && (!acc0 || !jerk0))
        return fail(FB_E_INVAL, "acc0 and jerk0 are required");
    if (N && (!finite_all(acc0, 3 * N) || !finite_all(jerk0, 3 * N)))
        return fail(FB_E_INVAL, "acc0 and jerk0 must be finite");
    for (size_t k = 0; k < ns; ++k) {
        if (dt_next && !(std::isfinite(dt_next[k]) && dt_next[k] >= 0.0))
            return fail(FB_E_INVAL, "dt_next[%zu] must be finite and >= 0", k);
        if (status && (status[k] < FB_SYS_ACTIVE || status[k] > FB_SYS_MAXSTEPS))
            return fail(FB_E_INVAL, "status[%zu] must be a Hermite status (0..%d)", k,
                        FB_SYS_MAXSTEPS);
        if (steps && steps[k] < 0)
            return fail(FB_E_INVAL, "steps[%zu] must be >= 0", k);
    }
    fb_ensemble *e = nullptr;
    fb_status st = fb_ensemble_create(n_sys, n_body, mass, pos, vel, t, hip_stream, &e);
    if (st != FB_OK)
        return st;
    if (ns) {
        // stage acc | jerk | dt_next | steps | status (fits the input staging)
        std::vector<double> dtn(ns, 0.0);
        std::vector<long long> stp(ns, 0);
        std::vector<int> sts(ns, FB_SYS_DONE);
        for (size_t k = 0; k < ns; ++k) {
            if (dt_next)
                dtn[k] = dt_next[k];
            if (steps)
                stp[k] = steps[k];
            if (status)
                sts[k] = status[k];
        }
        double *d_acc = e->d_staging, *d_jerk = d_acc + 3 * N, *d_dtn = d_jerk + 3 * N;
        long long *d_steps = (long long *)(d_dtn + ns);
        int *d_status = (int *)(d_steps + ns);
        hipError_t err = hipMemcpyAsync(d_acc, acc0, 24 * N, hipMemcpyHostToDevice, e->stream);
        if (err == hipSuccess)
            err = hipMemcpyAsync(d_jerk, jerk0, 24 * N, hipMemcpyHostToDevice, e->stream);
        if (err == hipSuccess)
            err = hipMemcpyAsync(d_dtn, dtn.data(), 8 * ns, hipMemcpyHostToDevice, e->stream);
        if (err == hipSuccess)
            err = hipMemcpyAsync(d_steps, stp.data(), 8 * ns, hipMemcpyHostToDevice, e->stream);
        if (err == hipSuccess)
            err = hipMemcpyAsync(d_status, sts.data(), 4 * ns, hipMemcpyHostToDevice, e->stream);
        for (size_t b = 0; err == hipSuccess && b < e->buckets.size(); ++b)
            err = launch_restore(e->buckets[b], e->d_orig_off, d_acc, d_jerk, d_dtn, d_steps,
                                 d_status, e->stream);
        if (err == hipSuccess)
            err = hipStreamSynchronize(e->stream);   // the host vectors die at return
        if (err != hipSuccess) {
            free_ensemble(e);
            return hip_fail(err, "checkpoint restore");
        }
    }
    *out = e;
    return FB_OK;
}

fb_status fb_eval_rsqrt(const double *d_in, double *d_out, int64_t n, void *hip_stream)
{
    if (n < 0 || (n > 0 && (!d_in || !d_out)))
        return fail(FB_E_INVAL, "n must be >= 0 and d_in, d_out device pointers");
    FB_HIP(launch_rsqrt(d_in, d_out, (long long)n, (hipStream_t)hip_stream));
    return FB_OK;
}

fb_status fb_integrate_steps(fb_ensemble *e, int64_t n_steps, double dt, const fb_opts *po)
{
    if (!e)
        return fail(FB_E_INVAL, "ensemble is NULL");
    fb_opts o;
    fb_opts_default(&o);
    if (po)
        o = *po;
    if (o.adaptive)
        return fail(FB_E_INVAL, "fb_integrate_steps takes fixed steps (opts.adaptive must be 0)");
    if (n_steps < 0)
        return fail(FB_E_INVAL, "n_steps must be >= 0");
    if (!(std::isfinite(dt) && dt != 0.0))
        return fail(FB_E_INVAL, "dt must be finite and non-zero");
    fb_status st = check_opts(o);
    if (st != FB_OK)
        return st;
    st = check_large(e, o);
    if (st != FB_OK)
        return st;
    if (n_steps == 0 || e->n_sys == 0)
        return FB_OK;
    st = ensure_inertial(e);
    if (st != FB_OK)
        return st;
    for (const Bucket &B : e->buckets)
        FB_HIP(launch_begin_run(B, 1, n_steps, 0.0, dt, 0, 0.0, e->stream));
    return run(e, o, o.stop_rules ? -1 : n_steps);
}

fb_status fb_integrate_mvs(fb_ensemble *e, int64_t n_steps, double dt, const fb_opts *po)
{
    if (!e)
        return fail(FB_E_INVAL, "ensemble is NULL");
    fb_opts o;
    fb_opts_default(&o);
    if (po)
        o = *po;
    if (o.adaptive || o.stop_rules || o.compact || o.schedule != FB_SCHED_PLAIN)
        return fail(FB_E_INVAL, "MVS takes fixed steps on the plain schedule without stop rules "
                                "(opts.adaptive, stop_rules and compact must be 0, schedule plain)");
    fb_status st = check_opts(o);
    if (st != FB_OK)
        return st;
    if (n_steps < 0)
        return fail(FB_E_INVAL, "n_steps must be >= 0");
    if (!(std::isfinite(dt) && dt != 0.0))
        return fail(FB_E_INVAL, "dt must be finite and non-zero");
    if (n_steps == 0 || e->n_sys == 0)
        return FB_OK;
    if (!e->mvs_form()) {
        for (const Bucket &B : e->buckets)
            FB_HIP(launch_mvs_enter(B, e->stream));
        e->form = fb_ensemble::FORM_MVS;
    }
    for (const Bucket &B : e->buckets)
        FB_HIP(launch_begin_run(B, 1, n_steps, 0.0, dt, 0, 0.0, e->stream));
    return run_mvs(e, o, n_steps);
}

size_t fb_log_bytes(int32_t n_sys, const int32_t *n_body, int32_t kind, int32_t max_records)
{
    if (n_sys < 0 || (n_sys > 0 && !n_body) || max_records < 1)
        return 0;
    size_t bodies = 0;
    for (int32_t s = 0; s < n_sys; ++s) {
        if (n_body[s] < 2 || n_body[s] > kMaxLargeBodies)
            return 0;
        bodies += (size_t)n_body[s];
    }
    const size_t R = (size_t)max_records;
    switch (kind) {
    case FB_LOG_STATE: return 8 * R * ((size_t)n_sys + 6 * bodies);
    case FB_LOG_RV: return 8 * R * 2 * (size_t)n_sys;
    case FB_LOG_ENERGY: return 8 * R * 5 * (size_t)n_sys;
    default: return 0;
    }
}

fb_status fb_integrate_steps_logged(fb_ensemble *e, int64_t n_steps, double dt, const fb_opts *po,
                                    const fb_log_spec *log, int32_t *n_records)
{
    if (!e || !log)
        return fail(FB_E_INVAL, "ensemble and log are required");
    if (n_records)
        *n_records = 0;
    fb_opts o;
    fb_opts_default(&o);
    if (po)
        o = *po;
    if (o.adaptive)
        return fail(FB_E_INVAL, "logged integration takes fixed steps (opts.adaptive must be 0)");
    if (o.schedule != FB_SCHED_PLAIN)
        return fail(FB_E_INVAL, "logged integration runs the plain schedule");
    fb_status st = check_opts(o);
    if (st != FB_OK)
        return st;
    st = check_large(e, o);
    if (st != FB_OK)
        return st;
    if (n_steps < 0 || !(std::isfinite(dt) && dt != 0.0))
        return fail(FB_E_INVAL, "n_steps must be >= 0 and dt finite and non-zero");
    if (log->every < 1)
        return fail(FB_E_INVAL, "log.every must be >= 1");
    const long long records = 1 + n_steps / log->every + (n_steps % log->every ? 1 : 0);
    double los[3];
    st = check_log(e, log, records, los);
    if (st != FB_OK)
        return st;
    if (e->n_sys == 0)
        return FB_OK;
    st = ensure_inertial(e);
    if (st != FB_OK)
        return st;
    double *out = static_cast<double *>(log->d_buffer);
    int k = 0;
    for (const Bucket &B : e->buckets)
        FB_HIP(launch_log(B, e->d_orig_off, log->kind, los, k, log->max_records, out, e->stream));
    ++k;
    if (n_steps > 0) {
        for (const Bucket &B : e->buckets)
            FB_HIP(launch_begin_run(B, 1, n_steps, 0.0, dt, 0, 0.0, e->stream));
        fb_opts oq = o;
        oq.steps_per_quantum = log->every;
        for (long long done = 0; done < n_steps; done += log->every) {
            st = run_plain(e, oq, log->every);
            if (st != FB_OK)
                return st;
            for (const Bucket &B : e->buckets)
                FB_HIP(launch_log(B, e->d_orig_off, log->kind, los, k, log->max_records, out,
                                  e->stream));
            ++k;
        }
    }
    if (n_records)
        *n_records = k;
    return FB_OK;
}

fb_status fb_integrate_to_times(fb_ensemble *e, int32_t n_times, const double *t_obs, double dt,
                                const fb_opts *po, const fb_log_spec *log, int32_t *n_records)
{
    if (!e || !log || !t_obs)
        return fail(FB_E_INVAL, "ensemble, times and log are required");
    if (n_records)
        *n_records = 0;
    fb_opts o;
    fb_opts_default(&o);
    if (po)
        o = *po;
    fb_status st = check_opts(o);
    if (st != FB_OK)
        return st;
    st = check_large(e, o);
    if (st != FB_OK)
        return st;
    if (!o.adaptive && !(std::isfinite(dt) && dt > 0.0))
        return fail(FB_E_INVAL, "dt must be finite and > 0 (the times increase)");
    if (n_times < 1)
        return fail(FB_E_INVAL, "n_times must be >= 1");
    for (int32_t k = 0; k < n_times; ++k)
        if (!std::isfinite(t_obs[k]) || (k > 0 && !(t_obs[k] > t_obs[k - 1])))
            return fail(FB_E_INVAL, "times must be finite and strictly increasing (index %d)", k);
    double los[3];
    st = check_log(e, log, n_times, los);
    if (st != FB_OK)
        return st;
    if (e->n_sys == 0)
        return FB_OK;
    st = ensure_inertial(e);
    if (st != FB_OK)
        return st;
    double *out = static_cast<double *>(log->d_buffer);
    const int rule = o.adaptive == 2 ? 2 : (o.adaptive ? 1 : 0);
    for (int32_t k = 0; k < n_times; ++k) {
        for (const Bucket &B : e->buckets)
            FB_HIP(launch_begin_run(B, 0, 0, t_obs[k], dt, rule, o.eta, e->stream));
        st = run(e, o, -1);
        if (st != FB_OK)
            return st;
        for (const Bucket &B : e->buckets)
            FB_HIP(launch_log(B, e->d_orig_off, log->kind, los, k, log->max_records, out,
                              e->stream));
    }
    if (n_records)
        *n_records = n_times;
    return FB_OK;
}

fb_status fb_integrate_rkck_steps(fb_ensemble *e, int64_t n_steps, double dt, const fb_opts *po)
{
    if (!e)
        return fail(FB_E_INVAL, "ensemble is NULL");
    fb_opts o;
    fb_opts_default(&o);
    if (po)
        o = *po;
    fb_status st = check_rk_opts(o);
    if (st != FB_OK)
        return st;
    if (n_steps < 0)
        return fail(FB_E_INVAL, "n_steps must be >= 0");
    if (!(std::isfinite(dt) && dt != 0.0))
        return fail(FB_E_INVAL, "dt must be finite and non-zero");
    if (n_steps == 0 || e->n_sys == 0)
        return FB_OK;
    st = ensure_xv(e);
    if (st != FB_OK)
        return st;
    for (const Bucket &B : e->buckets)
        FB_HIP(launch_begin_run(B, 1, n_steps, 0.0, dt, 0, 0.0, e->stream));
    e->form = fb_ensemble::FORM_XV;
    return run_rkck(e, o, 0, 0.0, n_steps);
}

fb_status fb_integrate_rkck(fb_ensemble *e, double t_end, double dt, double eps,
                            const fb_opts *po)
{
    if (!e)
        return fail(FB_E_INVAL, "ensemble is NULL");
    fb_opts o;
    fb_opts_default(&o);
    if (po)
        o = *po;
    fb_status st = check_rk_opts(o);
    if (st != FB_OK)
        return st;
    if (!std::isfinite(t_end))
        return fail(FB_E_INVAL, "t_end must be finite");
    if (!(std::isfinite(dt) && dt > 0.0))
        return fail(FB_E_INVAL, "dt (the first trial step) must be finite and > 0");
    if (!(std::isfinite(eps) && eps > 0.0))
        return fail(FB_E_INVAL, "eps must be finite and > 0");
    if (e->n_sys == 0)
        return FB_OK;
    st = ensure_xv(e);
    if (st != FB_OK)
        return st;
    for (const Bucket &B : e->buckets)
        FB_HIP(launch_begin_run(B, 0, 0, t_end, dt, 3, 0.0, e->stream));
    e->form = fb_ensemble::FORM_XV;
    return run_rkck(e, o, 3, eps, -1);
}

fb_status fb_integrate(fb_ensemble *e, double t_end, double dt, const fb_opts *po)
{
    if (!e)
        return fail(FB_E_INVAL, "ensemble is NULL");
    fb_opts o;
    fb_opts_default(&o);
    if (po)
        o = *po;
    fb_status st = check_opts(o);
    if (st != FB_OK)
        return st;
    st = check_large(e, o);
    if (st != FB_OK)
        return st;
    if (!std::isfinite(t_end))
        return fail(FB_E_INVAL, "t_end must be finite");
    if (!o.adaptive && !(std::isfinite(dt) && dt != 0.0))
        return fail(FB_E_INVAL, "dt must be finite and non-zero");
    if (e->n_sys == 0)
        return FB_OK;
    st = ensure_inertial(e);
    if (st != FB_OK)
        return st;
    for (const Bucket &B : e->buckets)
        FB_HIP(launch_begin_run(B, 0, 0, t_end, dt, o.adaptive == 2 ? 2 : (o.adaptive ? 1 : 0),
                                o.eta, e->stream));
    return run(e, o, -1);
}

fb_status fb_synchronize(fb_ensemble *e)
{
    if (!e)
        return fail(FB_E_INVAL, "ensemble is NULL");
    FB_HIP(hipStreamSynchronize(e->stream));
    return FB_OK;
}

fb_status fb_get_state(fb_ensemble *e, double *pos, double *vel, double *t, int32_t *status,
                       int64_t *steps)
{
    if (!e)
        return fail(FB_E_INVAL, "ensemble is NULL");
    const size_t N = (size_t)e->L.n_bodies, ns = (size_t)e->n_sys;
    if (ns == 0)
        return FB_OK;
    double *d_pos = e->d_staging, *d_vel = d_pos + 3 * N, *d_t = d_vel + 3 * N;
    long long *d_steps = (long long *)(d_t + ns);
    int *d_status = (int *)(d_steps + ns);
    for (const Bucket &B : e->buckets) {
        if (e->mvs_form())
            FB_HIP(launch_unpack_mvs(B, e->d_orig_off, pos ? d_pos : nullptr, vel ? d_vel : nullptr,
                                     t ? d_t : nullptr, status ? d_status : nullptr,
                                     steps ? d_steps : nullptr, e->stream));
        else
            FB_HIP(launch_unpack(B, e->d_orig_off, pos ? d_pos : nullptr, vel ? d_vel : nullptr,
                                 nullptr, nullptr, t ? d_t : nullptr, status ? d_status : nullptr,
                                 steps ? d_steps : nullptr, nullptr, e->stream));
    }
    if (pos)
        FB_HIP(hipMemcpyAsync(pos, d_pos, 24 * N, hipMemcpyDeviceToHost, e->stream));
    if (vel)
        FB_HIP(hipMemcpyAsync(vel, d_vel, 24 * N, hipMemcpyDeviceToHost, e->stream));
    if (t)
        FB_HIP(hipMemcpyAsync(t, d_t, 8 * ns, hipMemcpyDeviceToHost, e->stream));
    if (steps)
        FB_HIP(hipMemcpyAsync(steps, d_steps, 8 * ns, hipMemcpyDeviceToHost, e->stream));
    if (status)
        FB_HIP(hipMemcpyAsync(status, d_status, 4 * ns, hipMemcpyDeviceToHost, e->stream));
    FB_HIP(hipStreamSynchronize(e->stream));
    return FB_OK;
}

fb_status fb_get_hermite_state(fb_ensemble *e, double *acc0, double *jerk0, double *dt_next)
{
    if (!e)
        return fail(FB_E_INVAL, "ensemble is NULL");
    if (e->mvs_form())
        return fail(FB_E_STATE, "the ensemble holds MVS state; a Hermite integration restores "
                                "(a0, j0)");
    if (e->form == fb_ensemble::FORM_XV) {   // re-evaluate the stale (a0, j0)
        fb_status st = ensure_inertial(e);
        if (st != FB_OK)
            return st;
    }
    const size_t N = (size_t)e->L.n_bodies, ns = (size_t)e->n_sys;
    if (ns == 0)
        return FB_OK;
    double *d_acc = e->d_staging, *d_jerk = d_acc + 3 * N, *d_dtn = d_jerk + 3 * N;
    for (const Bucket &B : e->buckets)
        FB_HIP(launch_unpack(B, e->d_orig_off, nullptr, nullptr, acc0 ? d_acc : nullptr,
                             jerk0 ? d_jerk : nullptr, nullptr, nullptr, nullptr,
                             dt_next ? d_dtn : nullptr, e->stream));
    if (acc0)
        FB_HIP(hipMemcpyAsync(acc0, d_acc, 24 * N, hipMemcpyDeviceToHost, e->stream));
    if (jerk0)
        FB_HIP(hipMemcpyAsync(jerk0, d_jerk, 24 * N, hipMemcpyDeviceToHost, e->stream));
    if (dt_next)
        FB_HIP(hipMemcpyAsync(dt_next, d_dtn, 8 * ns, hipMemcpyDeviceToHost, e->stream));
    FB_HIP(hipStreamSynchronize(e->stream));
    return FB_OK;
}

fb_status fb_diagnostics(fb_ensemble *e, double *energy, double *angmom)
{
    if (!e)
        return fail(FB_E_INVAL, "ensemble is NULL");
    const size_t ns = (size_t)e->n_sys;
    if (ns == 0)
        return FB_OK;
    double *d_E = e->d_diag, *d_L = d_E + ns;
    for (const Bucket &B : e->buckets)
        FB_HIP(launch_diag(B, d_E, d_L, e->mvs_form(), e->stream));
    if (energy)
        FB_HIP(hipMemcpyAsync(energy, d_E, 8 * ns, hipMemcpyDeviceToHost, e->stream));
    if (angmom)
        FB_HIP(hipMemcpyAsync(angmom, d_L, 24 * ns, hipMemcpyDeviceToHost, e->stream));
    FB_HIP(hipStreamSynchronize(e->stream));
    return FB_OK;
}

fb_status fb_ensemble_shape(const fb_ensemble *e, int32_t *n_sys, int64_t *n_bodies)
{
    if (!e)
        return fail(FB_E_INVAL, "ensemble is NULL");
    if (n_sys)
        *n_sys = e->n_sys;
    if (n_bodies)
        *n_bodies = e->L.n_bodies;
    return FB_OK;
}

fb_status fb_ensemble_destroy(fb_ensemble *e)
{
    if (!e)
        return FB_OK;
    (void)hipStreamSynchronize(e->stream);
    free_ensemble(e);
    return FB_OK;
}

fb_status fb_set_plan(int32_t n, int32_t mapping, int32_t waves_per_group, int32_t groups_per_cu)
{
    if (n < 0 || n > kMaxBodies || n == 1)
        return fail(FB_E_INVAL, "plan index must be 0 (persistent launch) or 2..%d", kMaxBodies);
    if (mapping != FB_MAP_AUTO && mapping != FB_MAP_SYSTEM_PER_LANE &&
        mapping != FB_MAP_BODY_PER_LANE)
        return fail(FB_E_INVAL, "unknown mapping %d", mapping);
    if (waves_per_group < 1 || waves_per_group > 4)
        return fail(FB_E_INVAL, "waves_per_group must be 1..4");
    if (groups_per_cu < 0 || groups_per_cu > 32)
        return fail(FB_E_INVAL, "groups_per_cu must be 0..32");
    if (mapping == FB_MAP_SYSTEM_PER_LANE && n > 0 && n > kMaxSplBodies)
        return fail(FB_E_INVAL, "system-per-lane is built for n <= %d", kMaxSplBodies);
    std::lock_guard<std::mutex> lk(g_plan_mu);
    init_plans_locked();
    Plan &p = g_plan[n];
    p.mapping = mapping == FB_MAP_AUTO ? 0
                : mapping == FB_MAP_SYSTEM_PER_LANE ? MAP_SPL : MAP_BPL;
    p.waves_per_group = waves_per_group;
    p.groups_per_cu = groups_per_cu;
    return FB_OK;
}

fb_status fb_get_plan(int32_t n, int32_t *mapping, int32_t *waves_per_group,
                      int32_t *groups_per_cu)
{
    if (n < 0 || n > kMaxBodies || n == 1)
        return fail(FB_E_INVAL, "plan index must be 0 or 2..%d", kMaxBodies);
    const Plan p = get_plan(n);
    if (mapping)
        *mapping = p.mapping == MAP_SPL ? FB_MAP_SYSTEM_PER_LANE
                   : p.mapping == MAP_BPL ? FB_MAP_BODY_PER_LANE : FB_MAP_AUTO;
    if (waves_per_group)
        *waves_per_group = p.waves_per_group;
    if (groups_per_cu)
        *groups_per_cu = p.groups_per_cu;
    return FB_OK;
}

fb_status fb_autotune(fb_ensemble *e, int64_t steps, double dt, fb_tune_entry *out,
                      int32_t max_out, int32_t *n_out)
{
    if (!e)
        return fail(FB_E_INVAL, "ensemble is NULL");
    if (steps < 1 || !(std::isfinite(dt) && dt != 0.0))
        return fail(FB_E_INVAL, "steps must be >= 1 and dt finite, non-zero");
    if (n_out)
        *n_out = 0;
    if (e->n_sys == 0)
        return FB_OK;
    fb_status st0 = ensure_inertial(e);
    if (st0 != FB_OK)
        return st0;
    const size_t total = e->L.total;
    char *backup = nullptr;
    FB_HIP(hipStreamSynchronize(e->stream));
    FB_HIP(hipMalloc((void **)&backup, total));
    std::vector<fb_tune_entry> entries;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    fb_status result = FB_OK;
    auto run = [&]() -> fb_status {
        FB_HIP(hipEventCreate(&ev0));
        FB_HIP(hipEventCreate(&ev1));
        FB_HIP(hipMemcpyAsync(backup, e->base, total, hipMemcpyDeviceToDevice, e->stream));
        auto restore = [&]() -> hipError_t {
            return hipMemcpyAsync(e->base, backup, total, hipMemcpyDeviceToDevice, e->stream);
        };
        StepParams P;
        fb_opts o;
        fb_opts_default(&o);
        P = make_params(o, INT_MAX);
        // plain schedule: per bucket, mapping x waves per group (the large-n
        // buckets have a fixed launch shape and no plan to tune)
        for (const Bucket &B : e->buckets) {
            if (B.n > kMaxBodies)
                continue;
            struct Cand { int map, W; };
            std::vector<Cand> cands;
            for (int W : {1, 2, 4}) {
                if (B.n <= kMaxSplBodies)
                    cands.push_back({MAP_SPL, W});
                cands.push_back({MAP_BPL, W});
            }
            double best = 1e300;
            size_t best_i = 0;
            for (const Cand &c : cands) {
                FB_HIP(restore());
                FB_HIP(launch_begin_run(B, 1, 1, 0.0, dt, 0, 0.0, e->stream));
                FB_HIP(launch_plain(B, c.map, c.W, P, e->stream));   // warm-up (code load)
                FB_HIP(restore());
                FB_HIP(launch_begin_run(B, 1, steps, 0.0, dt, 0, 0.0, e->stream));
                FB_HIP(hipEventRecord(ev0, e->stream));
                FB_HIP(launch_plain(B, c.map, c.W, P, e->stream));
                FB_HIP(hipEventRecord(ev1, e->stream));
                FB_HIP(hipEventSynchronize(ev1));
                float ms = 0.0f;
                FB_HIP(hipEventElapsedTime(&ms, ev0, ev1));
                fb_tune_entry t;
                std::memset(&t, 0, sizeof t);
                t.n = B.n;
                t.mapping = c.map == MAP_SPL ? FB_MAP_SYSTEM_PER_LANE : FB_MAP_BODY_PER_LANE;
                t.waves_per_group = c.W;
                t.ms = ms;
                entries.push_back(t);
                if (ms < best) {
                    best = ms;
                    best_i = entries.size() - 1;
                }
            }
            entries[best_i].chosen = 1;
            const Plan cur = get_plan(B.n);
            fb_status st = fb_set_plan(B.n, entries[best_i].mapping, entries[best_i].waves_per_group,
                                       cur.groups_per_cu);
            if (st != FB_OK)
                return st;
        }
        // persistent launch: waves per group x groups per CU
        const Plan keep0 = get_plan(0);
        fb_opts po;
        fb_opts_default(&po);
        po.schedule = FB_SCHED_PERSISTENT;
        double best = 1e300;
        size_t best_i = 0;
        for (int cls : {0, 1})
        for (int W : {1, 2, 4}) {
            const int occ = persistent_max_groups_per_cu(0, cls, W);
            // powers of two, and the most groups that fit a CU at once
            std::vector<int> counts = {1, 2, 4, 8, 16, 32};
            if (occ > 0 && std::find(counts.begin(), counts.end(), occ) == counts.end())
                counts.push_back(occ);
            std::sort(counts.begin(), counts.end());
            for (int g : counts) {
                if (occ > 0 && g > occ)
                    continue;
                const int cmap = cls ? FB_MAP_SYSTEM_PER_LANE : FB_MAP_BODY_PER_LANE;
                fb_status st = fb_set_plan(0, cmap, W, g);
                if (st != FB_OK)
                    return st;
                FB_HIP(restore());
                for (const Bucket &B : e->buckets)
                    FB_HIP(launch_begin_run(B, 1, steps, 0.0, dt, 0, 0.0, e->stream));
                FB_HIP(hipEventRecord(ev0, e->stream));
                st = run_persistent(e, po, steps);
                if (st != FB_OK)
                    return st;
                FB_HIP(hipEventRecord(ev1, e->stream));
                FB_HIP(hipEventSynchronize(ev1));
                float ms = 0.0f;
                FB_HIP(hipEventElapsedTime(&ms, ev0, ev1));
                fb_tune_entry t;
                std::memset(&t, 0, sizeof t);
                t.n = 0;
                t.mapping = cmap;
                t.waves_per_group = W;
                t.groups_per_cu = g;
                t.ms = ms;
                entries.push_back(t);
                if (ms < best) {
                    best = ms;
                    best_i = entries.size() - 1;
                }
            }
        }
        (void)keep0;
        entries[best_i].chosen = 1;
        fb_status st = fb_set_plan(0, entries[best_i].mapping, entries[best_i].waves_per_group,
                                   entries[best_i].groups_per_cu);
        if (st != FB_OK)
            return st;
        FB_HIP(restore());
        FB_HIP(hipStreamSynchronize(e->stream));
        return FB_OK;
    };
    result = run();
    (void)hipStreamSynchronize(e->stream);
    if (ev0)
        (void)hipEventDestroy(ev0);
    if (ev1)
        (void)hipEventDestroy(ev1);
    (void)hipFree(backup);
    if (out)
        for (int32_t i = 0; i < max_out && i < (int32_t)entries.size(); ++i)
            out[i] = entries[i];
    if (n_out)
        *n_out = (int32_t)entries.size();
    return result;
}

fb_status fb_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_on = on != 0;
    return FB_OK;
}

fb_status fb_profile_read(double *kernel_ms, int64_t *launches)
{
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        ev.swap(g_prof_events);
    }
    double ms = 0.0;
    int64_t n = 0;
    for (auto &p : ev) {
        float f = 0.0f;
        if (hipEventSynchronize(p.second) == hipSuccess &&
            hipEventElapsedTime(&f, p.first, p.second) == hipSuccess) {
            ms += f;
            ++n;
        }
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    std::lock_guard<std::mutex> lk(g_prof_mu);
    g_prof_ms += ms;
    g_prof_launches += n;
    if (kernel_ms)
        *kernel_ms = g_prof_ms;
    if (launches)
        *launches = g_prof_launches;
    g_prof_ms = 0.0;
    g_prof_launches = 0;
    return FB_OK;
}

const char *fb_last_error(void) { return g_err; }

fb_status fb_fp64_fma_ceiling(double *tflops)
{
    if (!tflops)
        return fail(FB_E_INVAL, "tflops is NULL");
    *tflops = 0.0;
    int dev = 0;
    FB_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    FB_HIP(hipGetDeviceProperties(&prop, dev));
    const int cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    const int blocks = 8 * cu, iters = 20000;
    double *out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    fb_status st = FB_OK;
    hipError_t e = hipMalloc((void **)&out, sizeof(double) * 256 * (size_t)blocks);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipEventCreate(&a);
    if (e == hipSuccess)
        e = hipEventCreate(&b);
    float best_ms = 0.0f;
    for (int rep = 0; e == hipSuccess && rep < 3; ++rep) {
        e = hipEventRecord(a, s);
        if (e == hipSuccess)
            e = launch_fma_probe(out, blocks, iters, s);
        if (e == hipSuccess)
            e = hipEventRecord(b, s);
        if (e == hipSuccess)
            e = hipEventSynchronize(b);
        float ms = 0.0f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && rep > 0 && (best_ms == 0.0f || ms < best_ms))
            best_ms = ms;
    }
    if (e != hipSuccess)
        st = hip_fail(e, "FP64 FMA probe");
    else if (best_ms > 0.0f)
        *tflops = 2.0 * 16.0 * iters * 256.0 * blocks / (best_ms * 1e-3) / 1e12;
    if (a)
        (void)hipEventDestroy(a);
    if (b)
        (void)hipEventDestroy(b);
    if (s)
        (void)hipStreamDestroy(s);
    if (out)
        (void)hipFree(out);
    return st;
}

const char *fb_version(void) { return "fewbody-hip 0.1 (gfx950, FP64 Hermite P(EC)^2)"; }

}  // extern "C"
