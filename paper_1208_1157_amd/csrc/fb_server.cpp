// fb_server.cpp -- continuous-batching integration server behind fb_server_*.
//
// Requests (each an ensemble of systems with its own t_end and fixed dt) are
// queued by fb_server_submit from any thread.  One worker thread owns the
// GPU work and loops over quanta:
//   1. admit queued requests in arrival order while their device state fits
//      the memory budget (a first-fit arena carved from one allocation made
//      at creation) and the resident-request cap; upload, pack into bucket
//      SoA and run the set-up evaluation on the device;
//   2. one fused persistent launch advances every resident system by at
//      most steps_per_quantum steps (tiles never mix requests, largest work
//      first);
//   3. requests whose step count is reached are unpacked and copied back,
//      their completion time is stamped after the quantum's synchronisation,
//      and their arena blocks are released for the next admissions.
// A request that arrives while others run joins at the next quantum, so
// their work overlaps on the device; its own arithmetic does not depend on
// what else is resident.
#include "fb_runtime_internal.h"

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace fb;
using namespace fb::rt;

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device allocation; blocks are 256-aligned.
class Arena {
public:
    void reset(char *base, size_t size)
    {
        base_ = base;
        size_ = size;
        free_.clear();
        if (size)
            free_[0] = size;
        used_ = peak_ = 0;
    }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = align_up(std::max<size_t>(bytes, 256), 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const size_t rest = it->second - bytes;
                free_.erase(it);
                if (rest)
                    free_[off + bytes] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align_up(std::max<size_t>(bytes, 256), 256);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    char *base() const { return base_; }
    size_t size() const { return size_; }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

private:
    char *base_ = nullptr;
    size_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Request {
    int64_t id = 0;
    int32_t n_sys = 0;
    int64_t n_bodies = 0;
    std::vector<int32_t> n_body;
    std::vector<double> mass, pos, vel;
    double t_end = 0.0, dt = 0.0;
    int state = FB_REQ_QUEUED;
    bool cancel = false;
    Layout L;
    size_t arena_off = 0;
    bool has_block = false;
    std::vector<Bucket> buckets;
    std::vector<long long> off;
    std::vector<std::vector<int>> origins;
    long long total_steps = 0, done_steps = 0;
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
    std::vector<double> out_pos, out_vel, out_t;
    std::vector<int32_t> out_status;
    std::vector<int64_t> out_steps;
};

// Whole fixed steps and the total step count of a run from t0 to t_end,
// exactly as the device schedules them (whole steps while t0 + k dt stays
// within t_end, then one shortened step unless the remainder is below
// 1e-9 |dt|).
long long schedule_steps(double t0, double t_end, double dt)
{
    if (!((t_end - t0) * dt > 0.0))
        return 0;
    const double span = (t_end - t0) / dt;
    long long nf = span > 0.0 ? (long long)std::floor(span) : 0;
    while (nf > 0 && (std::fma((double)nf, dt, t0) - t_end) * dt > 0.0)
        --nf;
    const double rem = t_end - std::fma((double)nf, dt, t0);
    return nf + ((rem * dt > 1e-9 * dt * dt) ? 1 : 0);
}

double flops_per_system_step(int n) { return 116.0 * n * (n - 1) / 2 + 120.0 * n; }

}  // namespace

struct fb_server {
    fb_server_opts opts;
    int device = 0;
    int num_cu = 256;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *d_arena = nullptr;
    Arena arena;
    Bucket *d_buckets = nullptr;
    int cap_buckets = 0;
    Tile *d_tiles = nullptr;
    int cap_tiles = 0;
    int *d_ints = nullptr;   // [0] ntiles, [1] head, [2] scratch flag
    std::vector<Bucket> h_buckets;
    std::vector<Tile> h_tiles;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    fb_status worker_status = FB_OK;
    std::string worker_error;
    std::deque<Request *> queue;
    std::vector<Request *> resident;
    std::unordered_map<int64_t, std::unique_ptr<Request>> all;
    int64_t next_id = 1;
    fb_server_stats st;
    std::thread worker;
};

namespace {

fb_status admit_one(fb_server *S, Request *R)
{
    char *base = S->arena.base() + R->arena_off;
    R->buckets = bucket_views(base, R->L);
    const int ns = R->n_sys;
    const size_t N = (size_t)R->n_bodies;
    R->off.assign(ns + 1, 0);
    for (int s = 0; s < ns; ++s)
        R->off[s + 1] = R->off[s] + R->n_body[s];
    long long *d_off = reinterpret_cast<long long *>(base + R->L.orig_off);
    double *stg = reinterpret_cast<double *>(base + R->L.staging);
    int *d_flag = reinterpret_cast<int *>(base + R->L.ints);
    FB_HIP(hipMemcpyAsync(d_off, R->off.data(), sizeof(long long) * (ns + 1), hipMemcpyHostToDevice,
                          S->stream));
    FB_HIP(hipMemcpyAsync(stg, R->mass.data(), 8 * N, hipMemcpyHostToDevice, S->stream));
    FB_HIP(hipMemcpyAsync(stg + N, R->pos.data(), 24 * N, hipMemcpyHostToDevice, S->stream));
    FB_HIP(hipMemcpyAsync(stg + 4 * N, R->vel.data(), 24 * N, hipMemcpyHostToDevice, S->stream));
    R->origins.clear();
    for (const Bucket &B : R->buckets) {
        R->origins.push_back(slot_origins(R->n_body, B));
        FB_HIP(hipMemcpyAsync(B.orig, R->origins.back().data(), sizeof(int) * B.pitch,
                              hipMemcpyHostToDevice, S->stream));
    }
    for (const Bucket &B : R->buckets)
        FB_HIP(launch_pack(B, stg, stg + N, stg + 4 * N, nullptr, d_off, d_flag, S->stream));
    for (const Bucket &B : R->buckets)
        FB_HIP(launch_prepare(B, S->stream));
    for (const Bucket &B : R->buckets)
        FB_HIP(launch_begin_run(B, 0, 0, R->t_end, R->dt, 0, 0.0, S->stream));
    R->total_steps = schedule_steps(0.0, R->t_end, R->dt);
    R->done_steps = 0;
    return FB_OK;
}

fb_status finish_one(fb_server *S, Request *R)
{
    char *base = S->arena.base() + R->arena_off;
    const size_t N = (size_t)R->n_bodies, ns = (size_t)R->n_sys;
    const long long *d_off = reinterpret_cast<const long long *>(base + R->L.orig_off);
    double *stg = reinterpret_cast<double *>(base + R->L.staging);
    double *d_pos = stg, *d_vel = stg + 3 * N, *d_t = stg + 6 * N;
    long long *d_steps = reinterpret_cast<long long *>(d_t + ns);
    int *d_status = reinterpret_cast<int *>(d_steps + ns);
    for (const Bucket &B : R->buckets)
        FB_HIP(launch_unpack(B, d_off, d_pos, d_vel, nullptr, nullptr, d_t, d_status, d_steps,
                             nullptr, S->stream));
    R->out_pos.resize(3 * N);
    R->out_vel.resize(3 * N);
    R->out_t.resize(ns);
    R->out_status.resize(ns);
    R->out_steps.resize(ns);
    if (N) {
        FB_HIP(hipMemcpyAsync(R->out_pos.data(), d_pos, 24 * N, hipMemcpyDeviceToHost, S->stream));
        FB_HIP(hipMemcpyAsync(R->out_vel.data(), d_vel, 24 * N, hipMemcpyDeviceToHost, S->stream));
    }
    if (ns) {
        FB_HIP(hipMemcpyAsync(R->out_t.data(), d_t, 8 * ns, hipMemcpyDeviceToHost, S->stream));
        FB_HIP(hipMemcpyAsync(R->out_steps.data(), d_steps, 8 * ns, hipMemcpyDeviceToHost,
                              S->stream));
        FB_HIP(hipMemcpyAsync(R->out_status.data(), d_status, 4 * ns, hipMemcpyDeviceToHost,
                              S->stream));
    }
    return FB_OK;
}

fb_status ensure_capacity(fb_server *S, int nb, int nt)
{
    if (nb > S->cap_buckets) {
        if (S->d_buckets)
            FB_HIP(hipFree(S->d_buckets));
        S->cap_buckets = std::max(nb, 2 * S->cap_buckets);
        FB_HIP(hipMalloc((void **)&S->d_buckets, sizeof(Bucket) * S->cap_buckets));
    }
    if (nt > S->cap_tiles) {
        if (S->d_tiles)
            FB_HIP(hipFree(S->d_tiles));
        S->cap_tiles = std::max(nt, 2 * S->cap_tiles);
        FB_HIP(hipMalloc((void **)&S->d_tiles, sizeof(Tile) * S->cap_tiles));
    }
    return FB_OK;
}

// One quantum over every resident request.  Returns the requests it finished.
fb_status run_quantum(fb_server *S, std::vector<Request *> &finished, double &sys_steps)
{
    const int Q = S->opts.steps_per_quantum;
    struct Item {
        Tile t;
        double cost;
    };
    std::vector<Item> items;
    S->h_buckets.clear();
    sys_steps = 0.0;
    // The fused-kernel class is fixed by the plan (auto: body-per-lane), never
    // by the resident mix, so every request sees the same arithmetic alone
    // and among others.
    const Plan p0 = get_plan(0);
    const int cls = p0.mapping == MAP_SPL ? 1 : 0;
    const int spl_lim = persistent_spl_limit(cls, 0);
    for (Request *R : S->resident) {
        const long long left = R->total_steps - R->done_steps;
        const long long adv = std::min<long long>(left, Q);
        sys_steps += (double)R->n_sys * (double)adv;
        for (const Bucket &B : R->buckets) {
            const int bi = (int)S->h_buckets.size();
            S->h_buckets.push_back(B);
            const Plan p = get_plan(B.n);
            const int map = (B.n <= spl_lim && (p.mapping == MAP_SPL || cls == 1)) ? MAP_SPL : MAP_BPL;
            const int cap = tile_systems(map, B.n);
            for (int f = 0; f < B.count; f += cap) {
                Item it;
                it.t.bucket = bi;
                it.t.first = f;
                it.t.count = std::min(cap, B.count - f);
                it.t.kind = map * 32 + B.n;
                it.cost = (double)it.t.count * flops_per_system_step(B.n) * (double)adv;
                items.push_back(it);
            }
        }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const Item &a, const Item &b) { return a.cost > b.cost; });
    S->h_tiles.clear();
    for (const Item &it : items)
        S->h_tiles.push_back(it.t);
    const int nb = (int)S->h_buckets.size(), nt = (int)S->h_tiles.size();
    fb_status stc = ensure_capacity(S, nb, nt);
    if (stc != FB_OK)
        return stc;
    int ints[2] = {nt, 0};   // must outlive the asynchronous copy (synchronised below)
    if (nt > 0) {
        FB_HIP(hipMemcpyAsync(S->d_buckets, S->h_buckets.data(), sizeof(Bucket) * nb,
                              hipMemcpyHostToDevice, S->stream));
        FB_HIP(hipMemcpyAsync(S->d_tiles, S->h_tiles.data(), sizeof(Tile) * nt,
                              hipMemcpyHostToDevice, S->stream));
        FB_HIP(hipMemcpyAsync(S->d_ints, ints, sizeof ints, hipMemcpyHostToDevice, S->stream));
        StepParams P;
        P.adaptive = 0;
        P.stop_rules = 0;
        P.eta = 0.0;
        P.r_eject = 0.0;
        P.max_steps = LLONG_MAX;
        P.quantum = Q;
        P.pad = 0;
        const int W = std::max(1, std::min(4, p0.waves_per_group));
        int gpc = p0.groups_per_cu > 0 ? p0.groups_per_cu : 8;
        const int occ = persistent_max_groups_per_cu(0, cls, W);
        if (occ > 0)
            gpc = std::min(gpc, occ);
        const int grid = std::max(1, std::min(gpc * S->num_cu, nt));
        ProfScope ps(S->stream);
        FB_HIP(launch_persistent(S->d_buckets, S->d_tiles, S->d_ints, S->d_ints + 1, nullptr, P, 0,
                                 cls, grid, W, nullptr, S->stream));
    }
    for (Request *R : S->resident) {
        R->done_steps = std::min(R->total_steps, R->done_steps + Q);
        if (R->done_steps >= R->total_steps || R->cancel)
            finished.push_back(R);
    }
    for (Request *R : finished)
        if (!R->cancel) {
            fb_status s2 = finish_one(S, R);
            if (s2 != FB_OK)
                return s2;
        }
    FB_HIP(hipStreamSynchronize(S->stream));
    return FB_OK;
}

void worker_main(fb_server *S)
{
    (void)hipSetDevice(S->device);
    for (;;) {
        std::vector<Request *> admitted;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv_work.wait_for(lk, std::chrono::milliseconds(50), [&] {
                return S->stop || !S->queue.empty() || !S->resident.empty();
            });
            if (S->stop)
                break;
            // drop cancelled requests still in the queue
            for (auto it = S->queue.begin(); it != S->queue.end();) {
                if ((*it)->cancel) {
                    (*it)->state = FB_REQ_CANCELLED;
                    it = S->queue.erase(it);
                    S->cv_done.notify_all();
                } else {
                    ++it;
                }
            }
            // admission: arrival order, by memory budget and resident cap
            while (!S->queue.empty() &&
                   (int)(S->resident.size() + admitted.size()) < S->opts.max_resident) {
                Request *R = S->queue.front();
                size_t off = 0;
                if (!S->arena.alloc(R->L.total, off))
                    break;
                R->arena_off = off;
                R->has_block = true;
                S->queue.pop_front();
                admitted.push_back(R);
            }
        }
        fb_status err = FB_OK;
        for (Request *R : admitted) {
            err = admit_one(S, R);
            if (err != FB_OK)
                break;
        }
        std::vector<Request *> finished;
        double sys_steps = 0.0, t0 = now_s(), t1 = t0;
        if (err == FB_OK) {
            std::lock_guard<std::mutex> lk(S->mu);
            const double ta = now_s();
            for (Request *R : admitted) {
                R->state = FB_REQ_RUNNING;
                R->t_admit = ta;
                S->resident.push_back(R);
                S->st.admitted++;
            }
        }
        if (err == FB_OK && !S->resident.empty()) {
            t0 = now_s();
            err = run_quantum(S, finished, sys_steps);
            t1 = now_s();
        }
        std::lock_guard<std::mutex> lk(S->mu);
        if (err != FB_OK) {
            S->worker_status = err;
            S->worker_error = fb_last_error();
            for (auto &kv : S->all)
                if (kv.second->state == FB_REQ_QUEUED || kv.second->state == FB_REQ_RUNNING)
                    kv.second->state = FB_REQ_FAILED;
            S->queue.clear();
            S->resident.clear();
            S->cv_done.notify_all();
            break;
        }
        if (!S->resident.empty() || !finished.empty()) {
            S->st.quanta++;
            S->st.busy_seconds += t1 - t0;
            S->st.system_steps += sys_steps;
        }
        const double td = now_s();
        for (Request *R : finished) {
            R->t_done = td;
            R->state = R->cancel ? FB_REQ_CANCELLED : FB_REQ_DONE;
            if (!R->cancel)
                S->st.completed++;
            S->arena.release(R->arena_off, R->L.total);
            R->has_block = false;
            S->resident.erase(std::find(S->resident.begin(), S->resident.end(), R));
        }
        S->st.bytes_in_use = S->arena.used();
        S->st.peak_bytes = S->arena.peak();
        if (!finished.empty())
            S->cv_done.notify_all();
    }
}

bool finite_all(const double *p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i]))
            return false;
    return true;
}

}  // namespace

extern "C" {

void fb_server_opts_default(fb_server_opts *o)
{
    if (!o)
        return;
    std::memset(o, 0, sizeof *o);
    o->budget_bytes = (size_t)4 << 30;
    o->max_resident = 4096;
    o->steps_per_quantum = 2000;
}

double fb_monotonic_seconds(void) { return now_s(); }

fb_status fb_server_create(const fb_server_opts *po, void *hip_stream, fb_server **out)
{
    if (!out)
        return fail(FB_E_INVAL, "out is NULL");
    *out = nullptr;
    fb_server_opts o;
    fb_server_opts_default(&o);
    if (po) {
        if (po->budget_bytes)
            o.budget_bytes = po->budget_bytes;
        if (po->max_resident)
            o.max_resident = po->max_resident;
        if (po->steps_per_quantum)
            o.steps_per_quantum = po->steps_per_quantum;
    }
    if (o.max_resident < 1 || o.steps_per_quantum < 1 || o.budget_bytes < 4096)
        return fail(FB_E_INVAL, "max_resident and steps_per_quantum must be >= 1, budget >= 4 KiB");
    std::unique_ptr<fb_server> S(new fb_server());
    S->opts = o;
    std::memset(&S->st, 0, sizeof S->st);
    FB_HIP(hipGetDevice(&S->device));
    hipDeviceProp_t prop;
    FB_HIP(hipGetDeviceProperties(&prop, S->device));
    S->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    if (hip_stream) {
        S->stream = (hipStream_t)hip_stream;
    } else {
        FB_HIP(hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking));
        S->own_stream = true;
    }
    hipError_t e = hipMalloc((void **)&S->d_arena, o.budget_bytes);
    if (e != hipSuccess) {
        if (S->own_stream)
            (void)hipStreamDestroy(S->stream);
        return hip_fail(e, "hipMalloc(server budget)");
    }
    S->arena.reset(S->d_arena, o.budget_bytes);
    e = hipMalloc((void **)&S->d_ints, 64 * sizeof(int));
    if (e != hipSuccess) {
        (void)hipFree(S->d_arena);
        if (S->own_stream)
            (void)hipStreamDestroy(S->stream);
        return hip_fail(e, "hipMalloc(server control)");
    }
    fb_server *raw = S.release();
    raw->worker = std::thread(worker_main, raw);
    *out = raw;
    return FB_OK;
}

fb_status fb_server_submit(fb_server *S, int32_t n_sys, const int32_t *n_body, const double *mass,
                           const double *pos, const double *vel, double t_end, double dt,
                           int64_t *req_id)
{
    if (!S || !req_id)
        return fail(FB_E_INVAL, "server and req_id are required");
    std::unique_ptr<Request> R(new Request());
    if (!make_layout(n_sys, n_body, R->L))
        return fail(FB_E_INVAL, "n_sys must be >= 0 and every n_body in 2..%d", kMaxBodies);
    const size_t N = (size_t)R->L.n_bodies;
    if (N && (!mass || !pos || !vel))
        return fail(FB_E_INVAL, "mass, pos and vel are required");
    for (size_t i = 0; i < N; ++i)
        if (!(std::isfinite(mass[i]) && mass[i] >= 0.0))
            return fail(FB_E_INVAL, "mass[%zu] must be finite and >= 0", i);
    if (!finite_all(pos, 3 * N) || !finite_all(vel, 3 * N))
        return fail(FB_E_INVAL, "pos and vel must be finite");
    if (!(std::isfinite(t_end) && std::isfinite(dt) && dt != 0.0))
        return fail(FB_E_INVAL, "t_end must be finite and dt finite and non-zero");
    if (align_up(R->L.total, 256) > S->opts.budget_bytes)
        return fail(FB_E_BUDGET, "request needs %zu bytes of device state, budget is %zu",
                    R->L.total, S->opts.budget_bytes);
    R->n_sys = n_sys;
    R->n_bodies = (int64_t)N;
    R->n_body.assign(n_body, n_body + n_sys);
    R->mass.assign(mass, mass + N);
    R->pos.assign(pos, pos + 3 * N);
    R->vel.assign(vel, vel + 3 * N);
    R->t_end = t_end;
    R->dt = dt;
    R->t_submit = now_s();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->worker_status != FB_OK)
        return fail(S->worker_status, "server failed: %s", S->worker_error.c_str());
    R->id = S->next_id++;
    *req_id = R->id;
    S->queue.push_back(R.get());
    S->all[R->id] = std::move(R);
    S->st.submitted++;
    S->cv_work.notify_one();
    return FB_OK;
}

fb_status fb_server_poll(fb_server *S, int64_t req_id, int32_t *state)
{
    if (!S || !state)
        return fail(FB_E_INVAL, "server and state are required");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(req_id);
    if (it == S->all.end())
        return fail(FB_E_NOTFOUND, "unknown request %lld", (long long)req_id);
    *state = it->second->state;
    return FB_OK;
}

fb_status fb_server_wait(fb_server *S, int64_t req_id, double timeout_s, int32_t *state)
{
    if (!S)
        return fail(FB_E_INVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(req_id);
    if (it == S->all.end())
        return fail(FB_E_NOTFOUND, "unknown request %lld", (long long)req_id);
    Request *R = it->second.get();
    auto settled = [&] { return R->state >= FB_REQ_DONE; };
    if (timeout_s < 0)
        S->cv_done.wait(lk, settled);
    else
        S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), settled);
    if (state)
        *state = R->state;
    return FB_OK;
}

fb_status fb_server_result(fb_server *S, int64_t req_id, double *pos, double *vel, double *t,
                           int32_t *status, int64_t *steps, double *times)
{
    if (!S)
        return fail(FB_E_INVAL, "server is NULL");
    std::unique_ptr<Request> R;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(req_id);
        if (it == S->all.end())
            return fail(FB_E_NOTFOUND, "unknown request %lld", (long long)req_id);
        if (it->second->state != FB_REQ_DONE)
            return fail(FB_E_STATE, "request %lld is not done (state %d)", (long long)req_id,
                        it->second->state);
        R = std::move(it->second);
        S->all.erase(it);
    }
    const size_t N = (size_t)R->n_bodies, ns = (size_t)R->n_sys;
    if (pos && N)
        std::memcpy(pos, R->out_pos.data(), 24 * N);
    if (vel && N)
        std::memcpy(vel, R->out_vel.data(), 24 * N);
    if (t && ns)
        std::memcpy(t, R->out_t.data(), 8 * ns);
    if (status && ns)
        std::memcpy(status, R->out_status.data(), 4 * ns);
    if (steps && ns)
        std::memcpy(steps, R->out_steps.data(), 8 * ns);
    if (times) {
        times[0] = R->t_submit;
        times[1] = R->t_admit;
        times[2] = R->t_done;
    }
    return FB_OK;
}

fb_status fb_server_cancel(fb_server *S, int64_t req_id)
{
    if (!S)
        return fail(FB_E_INVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(req_id);
    if (it == S->all.end())
        return fail(FB_E_NOTFOUND, "unknown request %lld", (long long)req_id);
    if (it->second->state >= FB_REQ_DONE)
        return fail(FB_E_STATE, "request %lld already settled", (long long)req_id);
    it->second->cancel = true;
    S->cv_work.notify_one();
    return FB_OK;
}

fb_status fb_server_get_stats(fb_server *S, fb_server_stats *out)
{
    if (!S || !out)
        return fail(FB_E_INVAL, "server and stats are required");
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    out->queued = (int64_t)S->queue.size();
    out->resident = (int64_t)S->resident.size();
    out->bytes_in_use = S->arena.used();
    out->peak_bytes = S->arena.peak();
    if (S->worker_status != FB_OK)
        return fail(S->worker_status, "server failed: %s", S->worker_error.c_str());
    return FB_OK;
}

fb_status fb_server_destroy(fb_server *S)
{
    if (!S)
        return FB_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable())
        S->worker.join();
    (void)hipStreamSynchronize(S->stream);
    if (S->d_tiles)
        (void)hipFree(S->d_tiles);
    if (S->d_buckets)
        (void)hipFree(S->d_buckets);
    if (S->d_ints)
        (void)hipFree(S->d_ints);
    if (S->d_arena)
        (void)hipFree(S->d_arena);
    if (S->own_stream)
        (void)hipStreamDestroy(S->stream);
    delete S;
    return FB_OK;
}

}  // extern "C"
