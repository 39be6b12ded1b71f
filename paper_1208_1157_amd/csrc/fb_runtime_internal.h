// Host-runtime internals shared by fb_runtime.cpp (ensembles, plans, timing)
// and fb_server.cpp (continuous-batching server).  Not part of the ABI.
#pragma once

#include "fewbody.h"
#include "fb_internal.h"

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace fb {
namespace rt {

// Record an error message for fb_last_error() and return `code`.
fb_status fail(fb_status code, const char *fmt, ...);
fb_status hip_fail(hipError_t e, const char *what);

#define FB_HIP(call)                                  \
    do {                                              \
        hipError_t e_ = (call);                       \
        if (e_ != hipSuccess)                         \
            return ::fb::rt::hip_fail(e_, #call);     \
    } while (0)

struct Plan {
    int mapping;          // MAP_SPL / MAP_BPL (entry 0: fused-kernel class, 0 = auto)
    int waves_per_group;  // 1..4
    int groups_per_cu;    // persistent schedule only (entry 0)
};
Plan get_plan(int n);

// Lane mapping of a plain launch over bucket B: the plan's, or (auto)
// system-per-lane when n allows it and the bucket's 64-system tiles give
// every SIMD of the device a wavefront, else body-per-lane, whose n lanes
// per system spread a small bucket over more of the device.
inline int plain_mapping(const Plan &p, const Bucket &B, bool adv, int num_cu)
{
    const int lim = adv ? kMaxSplAdv : kMaxSplBodies;
    if (p.mapping == MAP_BPL || B.n > lim)
        return MAP_BPL;
    if (p.mapping == MAP_SPL)
        return MAP_SPL;
    return (B.count + 63) / 64 >= 4LL * num_cu ? MAP_SPL : MAP_BPL;
}

// Fused persistent kernel class for a launch over buckets of these body
// counts: the plan's choice, or (auto) for fixed steps the system-per-lane
// class when every bucket can run system-per-lane in it and its tiles (64
// systems each) give every SIMD of the device a wavefront; that class runs
// one wavefront per SIMD, so with fewer tiles the body-per-lane class, which
// spreads a system over n lanes, keeps more of the device busy.  With
// adaptive steps or stop rules (auto) always the body-per-lane class: a
// system-per-lane tile runs its 64 systems in lockstep, each to its own step
// count, and measured 1.7x slower than body-per-lane tiles (about 10
// systems each) on 65536 uneven-lifetime systems at full population.
template <class BucketRange>
int persistent_class(const Plan &p0, const BucketRange &buckets, bool adv, int num_cu)
{
    if (p0.mapping == MAP_SPL)
        return 1;
    if (p0.mapping == MAP_BPL || adv)
        return 0;
    const int lim = persistent_spl_limit(1, 0);
    long long tiles = 0;
    for (const Bucket &B : buckets) {
        if (B.n > lim)
            return 0;
        tiles += (B.count + 63) / 64;
    }
    return tiles >= 4LL * num_cu ? 1 : 0;
}

// Brackets the integration launches enqueued in its scope with HIP events on
// `s` when the kernel timer is enabled.
struct ProfScope {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t s;
    explicit ProfScope(hipStream_t st);
    ~ProfScope();
};

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Byte offsets of one body-count bucket inside an ensemble workspace.
struct BucketLayout {
    int n, count, pitch;
    size_t st, t, t_end, dt, dtn, t0run, krun, nfull, steps, status, orig;
};

// Device workspace of one ensemble: buckets in descending body count, then
// the tables, staging and scheduling arrays.
struct Layout {
    std::vector<BucketLayout> b;
    int64_t n_bodies = 0;
    int max_tiles = 0;
    int list_total = 0;
    size_t buckets, orig_off, staging, diag, ints, tiles, lists0, lists1, list_base, counts0,
        counts1, order, mapping, total;
};

bool make_layout(int32_t n_sys, const int32_t *n_body, Layout &L);
std::vector<Bucket> bucket_views(char *base, const Layout &L);
// Caller's system index of every slot of bucket B (padding slots -> 0).
std::vector<int> slot_origins(const std::vector<int32_t> &n_body, const Bucket &B);

}  // namespace rt
}  // namespace fb
