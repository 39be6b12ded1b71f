// fb_server.cpp -- continuous-batching integration server behind fb_server_*.
//
// Requests (each an ensemble of systems with its own t_end and fixed dt) are
// queued by fb_server_submit from any thread.  One worker thread owns the
// GPU work and loops over quanta:
//   1. admit queued requests in arrival order while their device state fits
//      the memory budget and the resident-request cap.  A request's systems
//      take free slots in the server-wide pool of their body count: chunks of
//      chunk_slots systems, each a bucket in the SoA layout, carved from one
//      allocation made at creation and returned when empty.  Its inputs are
//      uploaded, packed into those slots, and the set-up evaluation runs;
//   2. choose the requests this quantum advances (every resident one, or the
//      least remaining work first until the device is full), list their
//      slots chunk by chunk and cut the lists into tiles, so a tile holds
//      systems of several requests and stays full however small each request
//      is.  One fused persistent launch advances every listed system by at
//      most steps_per_quantum steps, costliest tiles first;
//   3. requests whose step count is reached are unpacked and copied back,
//      their completion time is stamped after the quantum's synchronisation,
//      and their slots and memory are released for the next admissions.
// A system's arithmetic depends only on its own state and on the kernel
// mapping its body count gets (fixed by the plan table), never on its slot,
// its tile, its neighbours or how its steps fall into quanta, so each
// request's results are the same alone and in any mix.
#include "fb_runtime_internal.h"

#include <algorithm>
#include <atomic>
#include <array>
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

// Device bytes of a pool chunk of `slots` systems of n bodies: the state rows
// and the per-system clock arrays, each 256-aligned.
size_t chunk_bytes(int n, int slots)
{
    const size_t P = (size_t)slots;
    return align_up(sizeof(double) * R_COUNT * n * P, 256) + 8 * align_up(8 * P, 256) +
           2 * align_up(4 * P, 256);
}

Bucket chunk_bucket(char *base, int n, int slots)
{
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char *p = base + o;
        o += align_up(bytes, 256);
        return p;
    };
    const size_t P = (size_t)slots;
    Bucket B;
    B.st = reinterpret_cast<double *>(take(sizeof(double) * R_COUNT * n * P));
    B.t = reinterpret_cast<double *>(take(8 * P));
    B.t_end = reinterpret_cast<double *>(take(8 * P));
    B.dt = reinterpret_cast<double *>(take(8 * P));
    B.dtn = reinterpret_cast<double *>(take(8 * P));
    B.t0run = reinterpret_cast<double *>(take(8 * P));
    B.krun = reinterpret_cast<long long *>(take(8 * P));
    B.nfull = reinterpret_cast<long long *>(take(8 * P));
    B.steps = reinterpret_cast<long long *>(take(8 * P));
    B.status = reinterpret_cast<int *>(take(4 * P));
    B.orig = reinterpret_cast<int *>(take(4 * P));
    B.n = n;
    B.pitch = slots;
    B.count = slots;
    B.pad = 0;
    return B;
}

// Slots first..first+count-1 of B as a bucket of their own: every per-slot
// array starts at `first`; the pitch (row stride) stays B's.
Bucket sub_view(const Bucket &B, int first, int count)
{
    Bucket v = B;
    v.st += first;
    v.t += first;
    v.t_end += first;
    v.dt += first;
    v.dtn += first;
    v.t0run += first;
    v.krun += first;
    v.nfull += first;
    v.steps += first;
    v.status += first;
    v.orig += first;
    v.count = count;
    return v;
}

// One chunk of a body-count pool, shared by the requests whose systems it
// holds.
struct Chunk {
    int n = 0;
    size_t off = 0, bytes = 0;
    Bucket B;                   // every slot: count == pitch
    std::map<int, int> free;    // free slot runs: first slot -> length
    int used = 0;
    int qidx = -1;              // index in the current quantum's bucket table
};

// A run of one request's slots in a chunk.
struct Piece {
    Chunk *c = nullptr;
    int first = 0, count = 0;
    std::vector<int> orig;      // caller's index of the system in each slot
    Bucket view() const { return sub_view(c->B, first, count); }
};

// Per-request device block: system offsets, and staging for the uploaded
// inputs (mass, pos, vel) and, later, the results (pos, vel, t, steps,
// status).
struct AuxLayout {
    size_t off_idx = 0, staging = 0, flag = 0, total = 0;
};

AuxLayout aux_layout(int64_t ns, int64_t N)
{
    AuxLayout A;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = align_up(o + std::max<size_t>(bytes, 1), 256);
        return r;
    };
    A.off_idx = take(8 * (size_t)(ns + 1));
    A.staging = take(8 * (size_t)std::max<int64_t>(7 * N, 6 * N + 2 * ns) + 4 * (size_t)ns);
    A.flag = take(64);
    A.total = o;
    return A;
}

struct Request {
    int64_t id = 0;
    int32_t n_sys = 0;
    int64_t n_bodies = 0;
    std::vector<int32_t> n_body;
    std::vector<double> mass, pos, vel;
    std::array<int, kMaxBodies + 1> cnt{};
    double t_end = 0.0, dt = 0.0;
    int state = FB_REQ_QUEUED;
    // set by fb_server_cancel (under the server lock), read by the worker
    // between quanta without it
    std::atomic<bool> cancel{false};
    AuxLayout aux;
    size_t aux_off = 0;
    bool has_aux = false;
    std::vector<Piece> pieces;
    std::vector<long long> off;
    long long total_steps = 0, done_steps = 0;
    double flops_per_step = 0.0;   // all its systems, one step each
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

// Relative duration of one step of a tile, in units of one pair: a
// system-per-lane lane walks all n(n-1)/2 pairs, a body-per-lane lane its
// n-1 partners.  The per-body and per-lane overheads are fitted to single-tile
// step times (3 and 10 bodies per lane: 0.69 and 9.3 us; 10 bodies, one body
// per lane: 2.4 us).
double tile_step_cost(int map, int n)
{
    return map == MAP_SPL ? 0.5 * n * (n - 1) + 0.15 * n : 1.2 * n;
}

// Device bytes a request needs on an empty server.
size_t request_bytes(const std::array<int, kMaxBodies + 1> &cnt, int64_t ns, int64_t N, int slots)
{
    size_t b = align_up(aux_layout(ns, N).total, 256);
    for (int n = 2; n <= kMaxBodies; ++n)
        if (cnt[n])
            b += (size_t)((cnt[n] + slots - 1) / slots) * align_up(chunk_bytes(n, slots), 256);
    return b;
}

}  // namespace

struct fb_server {
    fb_server_opts opts;
    int device = 0;
    int num_cu = 256;
    // Kernel mapping, fixed at creation from the plan table (entry 0's class,
    // auto meaning body-per-lane; per-n mappings), so a request's arithmetic
    // never depends on what else is resident or on later plan changes.
    int cls = 0, waves_per_group = 2, groups_per_cu = 8;
    int mapping[kMaxBodies + 1] = {0};
    hipStream_t stream = nullptr;
    bool own_stream = false;
    char *d_arena = nullptr;
    Arena arena;
    std::vector<std::unique_ptr<Chunk>> pool[kMaxBodies + 1];
    Bucket *d_buckets = nullptr;
    int cap_buckets = 0;
    Tile *d_tiles = nullptr;
    int cap_tiles = 0;
    int *d_list = nullptr;
    size_t cap_list = 0;
    int *d_ints = nullptr;   // [0] ntiles, [1] head
    std::vector<Bucket> h_buckets;
    std::vector<Tile> h_tiles;
    std::vector<int> h_list;

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

// Return a request's slots to their chunks, and empty chunks to the arena.
void release_pieces(fb_server *S, std::vector<Piece> &pieces)
{
    for (Piece &p : pieces) {
        Chunk *c = p.c;
        auto it = c->free.emplace(p.first, p.count).first;
        auto nx = std::next(it);
        if (nx != c->free.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            c->free.erase(nx);
        }
        if (it != c->free.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                c->free.erase(it);
            }
        }
        c->used -= p.count;
        if (c->used == 0) {
            S->arena.release(c->off, c->bytes);
            auto &pool = S->pool[c->n];
            pool.erase(std::find_if(pool.begin(), pool.end(),
                                    [c](const std::unique_ptr<Chunk> &q) { return q.get() == c; }));
        }
    }
    pieces.clear();
}

// k slots of the n-body pool: one free run that holds them all if there is
// one (first fit), else the free runs in chunk order, else new chunks.
// false (nothing taken beyond `out`, which the caller releases) when the
// arena cannot hold another chunk.
bool alloc_slots(fb_server *S, int n, int k, std::vector<Piece> &out)
{
    auto &pool = S->pool[n];
    auto take = [&](Chunk *c, std::map<int, int>::iterator it, int m) {
        const int first = it->first, len = it->second;
        c->free.erase(it);
        if (len > m)
            c->free.emplace(first + m, len - m);
        c->used += m;
        Piece p;
        p.c = c;
        p.first = first;
        p.count = m;
        out.push_back(std::move(p));
    };
    for (auto &cp : pool)
        for (auto it = cp->free.begin(); it != cp->free.end(); ++it)
            if (it->second >= k) {
                take(cp.get(), it, k);
                return true;
            }
    for (auto &cp : pool) {
        while (k > 0 && !cp->free.empty()) {
            const int m = std::min(k, cp->free.begin()->second);
            take(cp.get(), cp->free.begin(), m);
            k -= m;
        }
        if (k == 0)
            return true;
    }
    const int slots = S->opts.chunk_slots;
    while (k > 0) {
        std::unique_ptr<Chunk> c(new Chunk());
        c->n = n;
        c->bytes = chunk_bytes(n, slots);
        if (!S->arena.alloc(c->bytes, c->off))
            return false;
        c->B = chunk_bucket(S->arena.base() + c->off, n, slots);
        c->free.emplace(0, slots);
        Chunk *raw = c.get();
        pool.push_back(std::move(c));
        const int m = std::min(k, slots);
        take(raw, raw->free.begin(), m);
        k -= m;
    }
    return true;
}

// Memory for a queued request: its aux block and slots for all its systems.
// On failure everything taken is given back.
bool reserve(fb_server *S, Request *R)
{
    if (!S->arena.alloc(R->aux.total, R->aux_off))
        return false;
    R->has_aux = true;
    std::vector<std::vector<int>> by_n(kMaxBodies + 1);
    for (int s = 0; s < R->n_sys; ++s)
        by_n[R->n_body[s]].push_back(s);
    for (int n = kMaxBodies; n >= 2; --n) {
        if (by_n[n].empty())
            continue;
        const size_t before = R->pieces.size();
        if (!alloc_slots(S, n, (int)by_n[n].size(), R->pieces)) {
            release_pieces(S, R->pieces);
            S->arena.release(R->aux_off, R->aux.total);
            R->has_aux = false;
            return false;
        }
        size_t k = 0;
        for (size_t i = before; i < R->pieces.size(); ++i) {
            Piece &p = R->pieces[i];
            p.orig.assign(by_n[n].begin() + k, by_n[n].begin() + k + p.count);
            k += p.count;
        }
    }
    return true;
}

// Free a request's host copies of its inputs (once its uploads completed),
// and with `outputs` its host results too.
void drop_payload(Request *R, bool outputs)
{
    std::vector<double>().swap(R->mass);
    std::vector<double>().swap(R->pos);
    std::vector<double>().swap(R->vel);
    if (outputs) {
        std::vector<double>().swap(R->out_pos);
        std::vector<double>().swap(R->out_vel);
        std::vector<double>().swap(R->out_t);
        std::vector<int32_t>().swap(R->out_status);
        std::vector<int64_t>().swap(R->out_steps);
    }
}

void release_request(fb_server *S, Request *R)
{
    release_pieces(S, R->pieces);
    if (R->has_aux) {
        S->arena.release(R->aux_off, R->aux.total);
        R->has_aux = false;
    }
}

fb_status admit_one(fb_server *S, Request *R)
{
    char *aux = S->arena.base() + R->aux_off;
    const int ns = R->n_sys;
    const size_t N = (size_t)R->n_bodies;
    R->off.assign(ns + 1, 0);
    for (int s = 0; s < ns; ++s)
        R->off[s + 1] = R->off[s] + R->n_body[s];
    long long *d_off = reinterpret_cast<long long *>(aux + R->aux.off_idx);
    double *stg = reinterpret_cast<double *>(aux + R->aux.staging);
    int *d_flag = reinterpret_cast<int *>(aux + R->aux.flag);
    FB_HIP(hipMemcpyAsync(d_off, R->off.data(), sizeof(long long) * (ns + 1), hipMemcpyHostToDevice,
                          S->stream));
    if (N) {
        FB_HIP(hipMemcpyAsync(stg, R->mass.data(), 8 * N, hipMemcpyHostToDevice, S->stream));
        FB_HIP(hipMemcpyAsync(stg + N, R->pos.data(), 24 * N, hipMemcpyHostToDevice, S->stream));
        FB_HIP(hipMemcpyAsync(stg + 4 * N, R->vel.data(), 24 * N, hipMemcpyHostToDevice, S->stream));
    }
    for (const Piece &p : R->pieces) {
        const Bucket V = p.view();
        FB_HIP(hipMemcpyAsync(V.orig, p.orig.data(), sizeof(int) * p.count, hipMemcpyHostToDevice,
                              S->stream));
        FB_HIP(launch_pack(V, stg, stg + N, stg + 4 * N, nullptr, d_off, d_flag, false, S->stream));
        FB_HIP(launch_prepare(V, S->stream));
        FB_HIP(launch_begin_run(V, 0, 0, R->t_end, R->dt, 0, 0.0, S->stream));
    }
    R->total_steps = schedule_steps(0.0, R->t_end, R->dt);
    R->done_steps = 0;
    return FB_OK;
}

fb_status finish_one(fb_server *S, Request *R)
{
    char *aux = S->arena.base() + R->aux_off;
    const size_t N = (size_t)R->n_bodies, ns = (size_t)R->n_sys;
    const long long *d_off = reinterpret_cast<const long long *>(aux + R->aux.off_idx);
    double *stg = reinterpret_cast<double *>(aux + R->aux.staging);
    double *d_pos = stg, *d_vel = stg + 3 * N, *d_t = stg + 6 * N;
    long long *d_steps = reinterpret_cast<long long *>(d_t + ns);
    int *d_status = reinterpret_cast<int *>(d_steps + ns);
    for (const Piece &p : R->pieces)
        FB_HIP(launch_unpack(p.view(), d_off, d_pos, d_vel, nullptr, nullptr, d_t, d_status,
                             d_steps, nullptr, S->stream));
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

template <class T>
fb_status grow(T *&p, size_t &cap, size_t need)
{
    if (need <= cap)
        return FB_OK;
    if (p)
        FB_HIP(hipFree(p));
    p = nullptr;
    cap = std::max(need, 2 * cap);
    FB_HIP(hipMalloc((void **)&p, sizeof(T) * cap));
    return FB_OK;
}

// Fused-kernel mapping of body count n under class cls.
int server_mapping(const fb_server *S, int n)
{
    const int lim = persistent_spl_limit(S->cls, 0);
    // an explicit body-per-lane plan wins over the class's system-per-lane default
    return (n <= lim && S->mapping[n] != MAP_BPL && (S->mapping[n] == MAP_SPL || S->cls == 1))
               ? MAP_SPL : MAP_BPL;
}

// One quantum.  Returns the requests it finished (reached their step count
// or were cancelled).
fb_status run_quantum(fb_server *S, std::vector<Request *> &finished, double &sys_steps,
                      bool &spread)
{
    spread = false;
    const int Q = S->opts.steps_per_quantum;
    sys_steps = 0.0;
    const int cls = S->cls, W = S->waves_per_group, gpc = S->groups_per_cu;

    std::vector<Request *> live;
    for (Request *R : S->resident) {
        if (R->cancel || R->done_steps >= R->total_steps)
            finished.push_back(R);
        else
            live.push_back(R);
    }
    // Requests this quantum advances.
    std::vector<Request *> sched;
    if (S->opts.policy == FB_POLICY_SRPT) {
        std::stable_sort(live.begin(), live.end(), [](const Request *a, const Request *b) {
            return (double)(a->total_steps - a->done_steps) * a->flops_per_step <
                   (double)(b->total_steps - b->done_steps) * b->flops_per_step;
        });
        const long long target = S->opts.quantum_tiles > 0
                                     ? S->opts.quantum_tiles
                                     : 2LL * gpc * W * S->num_cu;
        auto tiles_of = [&](const Request *R) {
            long long t = 0;
            for (int n = 2; n <= kMaxBodies; ++n)
                if (R->cnt[n]) {
                    const int cap = tile_systems(server_mapping(S, n), n);
                    t += (R->cnt[n] + cap - 1) / cap;
                }
            return t;
        };
        // Long requests run every quantum and do not count against the
        // target: it bounds only the part chosen by remaining work.
        const long long L = S->opts.long_steps;
        long long tiles = 0;
        std::vector<Request *> rest;
        for (Request *R : live) {
            if (L > 0 && R->total_steps - R->done_steps >= L)
                sched.push_back(R);
            else
                rest.push_back(R);
        }
        for (Request *R : rest) {
            if (tiles >= target)
                break;
            sched.push_back(R);
            tiles += tiles_of(R);
        }
    } else {
        sched = live;
    }

    // Slot runs of the scheduled requests, grouped by chunk (largest n
    // first) and, inside a chunk, by steps left this quantum so that a tile's
    // lanes finish together.
    struct Run {
        Chunk *c;
        int first, count;
        long long adv;
    };
    std::vector<Run> runs;
    for (Request *R : sched) {
        const long long adv = std::min<long long>(R->total_steps - R->done_steps, Q);
        sys_steps += (double)R->n_sys * (double)adv;
        for (const Piece &p : R->pieces)
            runs.push_back({p.c, p.first, p.count, adv});
    }
    std::sort(runs.begin(), runs.end(), [](const Run &a, const Run &b) {
        if (a.c->n != b.c->n)
            return a.c->n > b.c->n;
        if (a.c != b.c)
            return a.c < b.c;
        if (a.adv != b.adv)
            return a.adv > b.adv;
        return a.first < b.first;
    });
    // One group of runs per chunk, with the mapping its tiles use.
    struct Group {
        size_t begin, end;
        int n, map;
        long long len, adv;   // systems; the most steps any of them takes this quantum
    };
    std::vector<Group> groups;
    for (size_t i = 0; i < runs.size();) {
        Group g{i, i, runs[i].c->n, server_mapping(S, runs[i].c->n), 0, runs[i].adv};
        for (; i < runs.size() && runs[i].c == runs[g.begin].c; ++i)
            g.len += runs[i].count;
        g.end = i;
        groups.push_back(g);
    }
    // A quantum lasts about as long as its slowest tile, or as its work spread
    // evenly over the resident waves if that is longer.  While it is the
    // slowest tile that sets the bound, the group with the slowest
    // system-per-lane tiles moves to body-per-lane tiles (n lanes per system,
    // each walking n-1 partners: more work, several times less time per
    // step), slowest first, as far as that lowers the bound.  A loaded quantum
    // keeps its mapping; a light one (a trace's tail, few requests) gets
    // shorter.  Both mappings give bitwise the same states, so a request's
    // results do not depend on it.
    const double resident_waves = (double)gpc * W * S->num_cu;
    if (cls == 1 && S->opts.idle_spread >= 0) {
        auto tiles = [&](const Group &G, int map) {
            const int cap = tile_systems(map, G.n);
            return (double)((G.len + cap - 1) / cap);
        };
        auto cost = [&](const Group &G, int map) {
            return (double)G.adv * tile_step_cost(map, G.n);
        };
        double work = 0.0, slow_bpl = 0.0;
        std::vector<size_t> order;
        for (size_t g = 0; g < groups.size(); ++g) {
            const Group &G = groups[g];
            work += tiles(G, G.map) * cost(G, G.map);
            if (G.map == MAP_SPL)
                order.push_back(g);
            else
                slow_bpl = std::max(slow_bpl, cost(G, MAP_BPL));
        }
        std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
            return cost(groups[a], MAP_SPL) > cost(groups[b], MAP_SPL);
        });
        // The prefix of `order` to move is the one with the lowest bound
        // (groups of equal cost only pay off together), if it gains at least
        // 5%: the extra work would otherwise be spent for little.
        auto bound = [&](double slowest, double w) { return std::max(slowest, w / resident_waves); };
        const size_t m = order.size();
        const double bound0 = bound(std::max(m ? cost(groups[order[0]], MAP_SPL) : 0.0, slow_bpl), work);
        double best = bound0;
        size_t best_k = 0;
        for (size_t k = 0; k < m; ++k) {
            const Group &G = groups[order[k]];
            work += tiles(G, MAP_BPL) * cost(G, MAP_BPL) - tiles(G, MAP_SPL) * cost(G, MAP_SPL);
            slow_bpl = std::max(slow_bpl, cost(G, MAP_BPL));
            const double next = k + 1 < m ? cost(groups[order[k + 1]], MAP_SPL) : 0.0;
            const double b = bound(std::max(next, slow_bpl), work);
            if (b < best) {
                best = b;
                best_k = k + 1;
            }
        }
        if (best > 0.95 * bound0)
            best_k = 0;
        for (size_t k = 0; k < best_k; ++k)
            groups[order[k]].map = MAP_BPL;
        spread = best_k > 0;
    }
    struct Item {
        Tile t;
        double cost;
    };
    std::vector<Item> items;
    S->h_buckets.clear();
    S->h_list.clear();
    for (const Group &G : groups) {
        Chunk *c = runs[G.begin].c;
        const int n = G.n;
        const int map = G.map;
        const int cap = tile_systems(map, n);
        const int bi = (int)S->h_buckets.size();
        S->h_buckets.push_back(c->B);
        const size_t list0 = S->h_list.size();
        std::vector<long long> adv_of;
        for (size_t i = G.begin; i < G.end; ++i)
            for (int k = 0; k < runs[i].count; ++k) {
                S->h_list.push_back(runs[i].first + k);
                adv_of.push_back(runs[i].adv);
            }
        const size_t len = S->h_list.size() - list0;
        for (size_t f = 0; f < len; f += cap) {
            Item it;
            it.t.bucket = bi;
            it.t.first = (int)(list0 + f);
            it.t.count = (int)std::min<size_t>(cap, len - f);
            it.t.kind = map * 32 + n;
            it.cost = (double)adv_of[f] * tile_step_cost(map, n);   // adv_of is non-increasing
            items.push_back(it);
        }
    }
    std::stable_sort(items.begin(), items.end(),
                     [](const Item &a, const Item &b) { return a.cost > b.cost; });
    S->h_tiles.clear();
    for (const Item &it : items)
        S->h_tiles.push_back(it.t);
    const int nb = (int)S->h_buckets.size(), nt = (int)S->h_tiles.size();
    size_t cb = (size_t)S->cap_buckets, ct = (size_t)S->cap_tiles;
    fb_status stc = grow(S->d_buckets, cb, (size_t)nb);
    if (stc == FB_OK)
        stc = grow(S->d_tiles, ct, (size_t)nt);
    if (stc == FB_OK)
        stc = grow(S->d_list, S->cap_list, S->h_list.size());
    S->cap_buckets = (int)cb;
    S->cap_tiles = (int)ct;
    if (stc != FB_OK)
        return stc;
    int ints[2] = {nt, 0};   // must outlive the asynchronous copy (synchronised below)
    if (nt > 0) {
        FB_HIP(hipMemcpyAsync(S->d_buckets, S->h_buckets.data(), sizeof(Bucket) * nb,
                              hipMemcpyHostToDevice, S->stream));
        FB_HIP(hipMemcpyAsync(S->d_tiles, S->h_tiles.data(), sizeof(Tile) * nt,
                              hipMemcpyHostToDevice, S->stream));
        FB_HIP(hipMemcpyAsync(S->d_list, S->h_list.data(), sizeof(int) * S->h_list.size(),
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
        const int grid = std::max(1, std::min(gpc * S->num_cu, nt));
        ProfScope ps(S->stream);
        FB_HIP(launch_persistent(S->d_buckets, S->d_tiles, S->d_ints, S->d_ints + 1, S->d_list, P,
                                 0, cls, grid, W, nullptr, S->stream));
    }
    for (Request *R : sched) {
        R->done_steps = std::min(R->total_steps, R->done_steps + Q);
        if (R->done_steps >= R->total_steps)
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
                    drop_payload(*it, true);
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
                if (!reserve(S, R))
                    break;
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
        bool spread = false;
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
            err = run_quantum(S, finished, sys_steps, spread);
            t1 = now_s();
        }
        if (err == FB_OK)   // the quantum synchronised: the admitted uploads are done
            for (Request *R : admitted)
                drop_payload(R, false);
        std::lock_guard<std::mutex> lk(S->mu);
        if (err != FB_OK) {
            S->worker_status = err;
            S->worker_error = fb_last_error();
            (void)hipStreamSynchronize(S->stream);
            for (auto &kv : S->all)
                if (kv.second->state == FB_REQ_QUEUED || kv.second->state == FB_REQ_RUNNING) {
                    kv.second->state = FB_REQ_FAILED;
                    drop_payload(kv.second.get(), true);
                }
            S->queue.clear();
            S->resident.clear();
            S->cv_done.notify_all();
            break;
        }
        if (sys_steps > 0.0 || !finished.empty()) {
            S->st.quanta++;
            S->st.busy_seconds += t1 - t0;
            S->st.system_steps += sys_steps;
            S->st.spread_quanta += spread ? 1 : 0;
        }
        const double td = now_s();
        for (Request *R : finished) {
            R->t_done = td;
            R->state = R->cancel ? FB_REQ_CANCELLED : FB_REQ_DONE;
            if (R->cancel)
                drop_payload(R, true);
            else
                S->st.completed++;
            release_request(S, R);
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

// Fill o's zero fields from the defaults and check it.
fb_status resolve_opts(const fb_server_opts *po, fb_server_opts &o)
{
    fb_server_opts_default(&o);
    if (po) {
        if (po->budget_bytes)
            o.budget_bytes = po->budget_bytes;
        if (po->max_resident)
            o.max_resident = po->max_resident;
        if (po->steps_per_quantum)
            o.steps_per_quantum = po->steps_per_quantum;
        o.policy = po->policy;
        o.quantum_tiles = po->quantum_tiles;
        o.long_steps = po->long_steps;
        o.idle_spread = po->idle_spread;
        if (po->chunk_slots)
            o.chunk_slots = po->chunk_slots;
    }
    if (o.max_resident < 1 || o.steps_per_quantum < 1 || o.budget_bytes < 4096)
        return fail(FB_E_INVAL, "max_resident and steps_per_quantum must be >= 1, budget >= 4 KiB");
    if (o.policy != FB_POLICY_FAIR && o.policy != FB_POLICY_SRPT)
        return fail(FB_E_INVAL, "policy must be FB_POLICY_FAIR or FB_POLICY_SRPT");
    if (o.quantum_tiles < 0 || o.long_steps < 0)
        return fail(FB_E_INVAL, "quantum_tiles and long_steps must be >= 0");
    if (o.idle_spread < -1 || o.idle_spread > 1)
        return fail(FB_E_INVAL, "idle_spread must be -1, 0 or 1");
    if (o.chunk_slots < 64 || o.chunk_slots > (1 << 20) || o.chunk_slots % 64)
        return fail(FB_E_INVAL, "chunk_slots must be a multiple of 64 in 64..2^20");
    return FB_OK;
}

// Body-count histogram of a request; false on a bad count.
bool count_bodies(int32_t n_sys, const int32_t *n_body, std::array<int, kMaxBodies + 1> &cnt,
                         int64_t &N)
{
    cnt.fill(0);
    N = 0;
    if (n_sys < 0 || (n_sys > 0 && !n_body))
        return false;
    for (int32_t s = 0; s < n_sys; ++s) {
        if (n_body[s] < 2 || n_body[s] > kMaxBodies)
            return false;
        cnt[n_body[s]]++;
        N += n_body[s];
    }
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
    o->policy = FB_POLICY_FAIR;
    o->quantum_tiles = 0;
    o->chunk_slots = 512;
}

size_t fb_server_request_bytes(const fb_server_opts *po, int32_t n_sys, const int32_t *n_body)
{
    fb_server_opts o;
    std::array<int, kMaxBodies + 1> cnt;
    int64_t N = 0;
    if (resolve_opts(po, o) != FB_OK || !count_bodies(n_sys, n_body, cnt, N))
        return 0;
    return request_bytes(cnt, n_sys, N, o.chunk_slots);
}

double fb_monotonic_seconds(void) { return now_s(); }

fb_status fb_server_create(const fb_server_opts *po, void *hip_stream, fb_server **out)
{
    if (!out)
        return fail(FB_E_INVAL, "out is NULL");
    *out = nullptr;
    fb_server_opts o;
    const fb_status so = resolve_opts(po, o);
    if (so != FB_OK)
        return so;
    std::unique_ptr<fb_server> S(new fb_server());
    S->opts = o;
    std::memset(&S->st, 0, sizeof S->st);
    FB_HIP(hipGetDevice(&S->device));
    hipDeviceProp_t prop;
    FB_HIP(hipGetDeviceProperties(&prop, S->device));
    S->num_cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    const Plan p0 = get_plan(0);
    S->cls = p0.mapping == MAP_SPL ? 1 : 0;
    S->waves_per_group = std::max(1, std::min(4, p0.waves_per_group));
    S->groups_per_cu = p0.groups_per_cu > 0 ? p0.groups_per_cu : 8;
    const int occ = persistent_max_groups_per_cu(0, S->cls, S->waves_per_group);
    if (occ > 0)
        S->groups_per_cu = std::min(S->groups_per_cu, occ);
    for (int n = 2; n <= kMaxBodies; ++n)
        S->mapping[n] = get_plan(n).mapping;
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
    int64_t nbod = 0;
    if (!count_bodies(n_sys, n_body, R->cnt, nbod))
        return fail(FB_E_INVAL, "n_sys must be >= 0 and every n_body in 2..%d", kMaxBodies);
    const size_t N = (size_t)nbod;
    if (N && (!mass || !pos || !vel))
        return fail(FB_E_INVAL, "mass, pos and vel are required");
    for (size_t i = 0; i < N; ++i)
        if (!(std::isfinite(mass[i]) && mass[i] >= 0.0))
            return fail(FB_E_INVAL, "mass[%zu] must be finite and >= 0", i);
    if (!finite_all(pos, 3 * N) || !finite_all(vel, 3 * N))
        return fail(FB_E_INVAL, "pos and vel must be finite");
    if (!(std::isfinite(t_end) && std::isfinite(dt) && dt != 0.0))
        return fail(FB_E_INVAL, "t_end must be finite and dt finite and non-zero");
    const size_t need = request_bytes(R->cnt, n_sys, nbod, S->opts.chunk_slots);
    if (need > S->opts.budget_bytes)
        return fail(FB_E_BUDGET, "request needs %zu bytes of device memory, budget is %zu", need,
                    S->opts.budget_bytes);
    R->aux = aux_layout(n_sys, nbod);
    for (int n = 2; n <= kMaxBodies; ++n)
        R->flops_per_step += R->cnt[n] * flops_per_system_step(n);
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

fb_status fb_server_release(fb_server *S, int64_t req_id)
{
    if (!S)
        return fail(FB_E_INVAL, "server is NULL");
    std::unique_ptr<Request> R;   // freed after the lock is released
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(req_id);
        if (it == S->all.end())
            return fail(FB_E_NOTFOUND, "unknown request %lld", (long long)req_id);
        // settled requests are in no worker list any more
        if (it->second->state < FB_REQ_DONE)
            return fail(FB_E_STATE, "request %lld is not settled (state %d)", (long long)req_id,
                        it->second->state);
        R = std::move(it->second);
        S->all.erase(it);
    }
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
    if (S->d_list)
        (void)hipFree(S->d_list);
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
