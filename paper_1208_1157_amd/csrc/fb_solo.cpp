// fb_solo.cpp -- stateless fixed-step Hermite integration of one homogeneous
// batch of systems held in the caller's device arrays.
//
// The batch (n_sys systems of n bodies, body-major rows as everywhere in the
// ABI) is packed into one structure-of-arrays bucket, given its set-up
// evaluation (Algorithm 1's "prepare"), advanced by a plain launch of the
// same kernels an ensemble uses (Eq. 3 predictor, Eq. 4 corrector twice per
// step as in Algorithm 2), and unpacked back in place.  Nothing is read back
// to the host and nothing outlives the call, so the call is pure stream
// work.  The bucket lives either in a caller workspace or, for callers that
// cannot allocate device memory, in a fixed per-device array of this file.
#include "fewbody.h"
#include "fb_internal.h"
#include "fb_runtime_internal.h"

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <mutex>

using namespace fb;
using namespace fb::rt;

namespace {

// Largest batch the allocation-free entry point takes: bucket, tables and
// flag of, e.g., 131072 three-body or 38000 sixteen-body systems.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

// The allocation-free entry point's bucket.  Host code never uses this name
// as an address: every device gets its own copy, whose address is looked up
// once per device (g_scratch_ptr).
static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices];

// Batches above this many systems are rejected before any size arithmetic.
constexpr int32_t kMaxSoloSystems = 1 << 26;

// Byte offsets of the batch's bucket, its body-offset table and its input
// flag inside a workspace; plain arithmetic (no heap).
struct SoloLayout {
    BucketLayout b;
    size_t orig_off, ints, total;
};

bool solo_layout(int32_t n_sys, int32_t n, SoloLayout &L)
{
    if (n_sys < 0 || n_sys > kMaxSoloSystems || n < 2 || n > kMaxBodies)
        return false;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes, 256);
        return o;
    };
    BucketLayout &bl = L.b;
    bl.n = n;
    bl.count = n_sys;
    bl.pitch = (int)align_up((size_t)n_sys, 64);
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
    L.orig_off = take(8 * (P + 1));
    L.ints = take(256);
    L.total = off;
    return true;
}

Bucket solo_view(char *base, const SoloLayout &L)
{
    const BucketLayout &bl = L.b;
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
    return B;
}

fb_status solo_check(int32_t n_sys, int32_t n, const double *d_mass, const double *d_pos,
                     const double *d_vel, int64_t n_steps, double dt, SoloLayout &L)
{
    if (!solo_layout(n_sys, n, L))
        return fail(FB_E_INVAL, "n_sys must be in 0..%d and n in 2..%d", kMaxSoloSystems,
                    kMaxBodies);
    if (n_sys > 0 && (!d_mass || !d_pos || !d_vel))
        return fail(FB_E_INVAL, "d_mass, d_pos and d_vel are required");
    if (n_steps < 0)
        return fail(FB_E_INVAL, "n_steps must be >= 0");
    if (n_steps > 0 && !(std::isfinite(dt) && dt != 0.0))
        return fail(FB_E_INVAL, "dt must be finite and non-zero");
    return FB_OK;
}

// Enqueue pack, set-up evaluation, n_steps fixed steps and unpack of the
// batch on stream s, with the bucket at `base`.  The steps use the plan of
// body count n and the same launch as an ensemble's plain schedule.
fb_status solo_run(char *base, const SoloLayout &L, const double *d_mass, double *d_pos,
                   double *d_vel, int32_t *d_status, int64_t n_steps, double dt, hipStream_t s,
                   bool timed)
{
    const Bucket B = solo_view(base, L);
    long long *orig_off = reinterpret_cast<long long *>(base + L.orig_off);
    int *bad = reinterpret_cast<int *>(base + L.ints);
    int dev = 0, num_cu = 0;
    FB_HIP(hipGetDevice(&dev));
    FB_HIP(hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    const Plan p = get_plan(B.n);
    StepParams P;
    P.adaptive = 0;
    P.stop_rules = 0;
    P.eta = 0.01;
    P.r_eject = 100.0;
    P.max_steps = LLONG_MAX;
    P.quantum = INT_MAX;
    P.pad = 0;
    const int map = plain_mapping(p, B, false, num_cu > 0 ? num_cu : 256);
    FB_HIP(launch_identity_tables(B, orig_off, bad, s));
    FB_HIP(launch_pack(B, d_mass, d_pos, d_vel, nullptr, orig_off, bad, true, s));
    FB_HIP(launch_prepare(B, s));
    if (n_steps > 0) {
        FB_HIP(launch_begin_run(B, 1, n_steps, 0.0, dt, 0, 0.0, s));
        if (timed) {
            ProfScope ps(s);
            FB_HIP(launch_plain(B, map, p.waves_per_group, P, s));
        } else {
            FB_HIP(launch_plain(B, map, p.waves_per_group, P, s));
        }
    }
    FB_HIP(launch_unpack(B, orig_off, d_pos, d_vel, nullptr, nullptr, nullptr, d_status, nullptr,
                         nullptr, s));
    return FB_OK;
}

// This device's copy of `scratch`, looked up on the first call on the device
// (with the device current) and kept for the process.
fb_status device_scratch(char *&out)
{
    int dev = 0;
    FB_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(FB_E_DEVICE, "device %d is beyond the %d devices the static scratch serves",
                    dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!ptr || reinterpret_cast<uintptr_t>(ptr) % 256)
            return fail(FB_E_DEVICE, "static scratch at an unusable address");
        g_scratch_ptr[dev] = static_cast<char *>(ptr);
    }
    out = g_scratch_ptr[dev];
    return FB_OK;
}

}  // namespace

extern "C" {

fb_status fb_hermite_steps_device(int32_t n_sys, int32_t n, const double *d_mass, double *d_pos,
                                  double *d_vel, int32_t *d_status, int64_t n_steps, double dt,
                                  void *d_workspace, size_t ws_bytes, void *hip_stream)
{
    SoloLayout L;
    fb_status st = solo_check(n_sys, n, d_mass, d_pos, d_vel, n_steps, dt, L);
    if (st != FB_OK)
        return st;
    if (n_sys == 0)
        return FB_OK;
    if (!d_workspace || ws_bytes < L.total)
        return fail(FB_E_NOMEM, "workspace of %zu bytes needed, %zu given", L.total, ws_bytes);
    if (reinterpret_cast<uintptr_t>(d_workspace) % 256)
        return fail(FB_E_INVAL, "workspace must be 256-byte aligned");
    return solo_run(static_cast<char *>(d_workspace), L, d_mass, d_pos, d_vel, d_status, n_steps,
                    dt, (hipStream_t)hip_stream, true);
}

fb_status fb_hermite_steps_device_noalloc(int32_t n_sys, int32_t n, const double *d_mass,
                                          double *d_pos, double *d_vel, int32_t *d_status,
                                          int64_t n_steps, double dt, void *hip_stream)
{
    SoloLayout L;
    fb_status st = solo_check(n_sys, n, d_mass, d_pos, d_vel, n_steps, dt, L);
    if (st != FB_OK)
        return st;
    if (n_sys == 0)
        return FB_OK;
    if (L.total > kScratchBytes)
        return fail(FB_E_NOMEM,
                    "%d systems of %d bodies need %zu bytes; the static scratch holds %zu "
                    "(use fb_hermite_steps_device with a workspace)",
                    n_sys, n, L.total, kScratchBytes);
    char *base = nullptr;
    st = device_scratch(base);
    if (st != FB_OK)
        return st;
    return solo_run(base, L, d_mass, d_pos, d_vel, d_status, n_steps, dt,
                    (hipStream_t)hip_stream, false);
}

size_t fb_hermite_steps_workspace_bytes(int32_t n_sys, int32_t n)
{
    SoloLayout L;
    return solo_layout(n_sys, n, L) ? L.total : 0;
}

}  // extern "C"
