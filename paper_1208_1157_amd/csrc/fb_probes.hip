// fb_probes.hip -- device measurement utilities that compute nothing of the
// method: the LDS streaming rates of whole-wavefront 16-byte reads and
// writes.  The body-per-lane kernels exchange every evaluation state through
// LDS; these two rates decide whether an exchange or the FP64 arithmetic
// around it bounds a design.
#include "fewbody.h"
#include "fb_internal.h"
#include "fb_runtime_internal.h"

#include <hip/hip_runtime.h>

using namespace fb::rt;

namespace {

constexpr int kProbeSlots = 1024;   // 16-byte slots: 16 KB of LDS per workgroup
constexpr int kProbeUnroll = 8;     // accesses per iteration, 64 slots apart
constexpr int kProbeIters = 4096;
constexpr int kProbeGroupsPerCu = 8;   // 8 x 16 KB = 128 KB of a CU's 160 KB

// Every lane reads slot base + u * 64 (u < 8) with base < 512, so a
// wavefront's 64 lanes touch 64 consecutive slots (no bank conflicts) and no
// index reaches kProbeSlots.  Two FP64 adds per read keep the reads live.
__global__ __launch_bounds__(256) void k_lds_read(double *out, int iters)
{
    __shared__ double2 L[kProbeSlots];
    const int tid = threadIdx.x;
    for (int i = tid; i < kProbeSlots; i += 256)
        L[i] = make_double2((double)i, (double)(i + 1));
    __syncthreads();
    double ax = 0.0, ay = 0.0;
    for (int it = 0; it < iters; ++it) {
        const int base = (it * 64 + tid) & 511;
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u) {
            const double2 q = L[base + u * 64];
            ax += q.x;
            ay += q.y;
        }
    }
    out[(size_t)blockIdx.x * 256 + tid] = ax + ay;
}

// The same slots written instead; one read after the barrier keeps them.
__global__ __launch_bounds__(256) void k_lds_write(double *out, int iters)
{
    __shared__ double2 L[kProbeSlots];
    const int tid = threadIdx.x;
    double x = (double)tid;
    for (int it = 0; it < iters; ++it) {
        const int base = (it * 64 + tid) & 511;
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u)
            L[base + u * 64] = make_double2(x, x);
        x += 1.0;
    }
    __syncthreads();
    out[(size_t)blockIdx.x * 256 + tid] = L[(tid * 7) & (kProbeSlots - 1)].x;
}

}  // namespace

extern "C" {

fb_status fb_lds_rates(double *read_gbs_per_cu, double *write_gbs_per_cu)
{
    if (!read_gbs_per_cu || !write_gbs_per_cu)
        return fail(FB_E_INVAL, "rate pointer is NULL");
    *read_gbs_per_cu = 0.0;
    *write_gbs_per_cu = 0.0;
    int dev = 0;
    FB_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    FB_HIP(hipGetDeviceProperties(&prop, dev));
    const int cu = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    const int blocks = kProbeGroupsPerCu * cu;
    double *out = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipMalloc((void **)&out, sizeof(double) * 256 * (size_t)blocks);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipEventCreate(&a);
    if (e == hipSuccess)
        e = hipEventCreate(&b);
    // bytes one launch moves: every lane, every iteration, 8 x 16 bytes
    const double bytes = 256.0 * blocks * kProbeIters * kProbeUnroll * 16.0;
    for (int kind = 0; kind < 2 && e == hipSuccess; ++kind) {
        float best_ms = 0.0f;
        for (int rep = 0; e == hipSuccess && rep < 3; ++rep) {   // the first is a warm-up
            e = hipEventRecord(a, s);
            if (e == hipSuccess) {
                if (kind == 0)
                    hipLaunchKernelGGL(k_lds_read, dim3(blocks), dim3(256), 0, s, out, kProbeIters);
                else
                    hipLaunchKernelGGL(k_lds_write, dim3(blocks), dim3(256), 0, s, out, kProbeIters);
                e = hipGetLastError();
            }
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
        if (e == hipSuccess && best_ms > 0.0f)
            *(kind == 0 ? read_gbs_per_cu : write_gbs_per_cu) = bytes / (best_ms * 1e-3) / cu / 1e9;
    }
    fb_status st = FB_OK;
    if (e != hipSuccess)
        st = hip_fail(e, "LDS probe");
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

}  // extern "C"
