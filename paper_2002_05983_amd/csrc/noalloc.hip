// noalloc.hip -- stencil_run without device allocation.
//
// stencil_run ping-pongs between the caller's output and the plan's scratch
// grid, which stencil_plan allocates.  stencil_run_noalloc runs the same
// kernels and pass schedule with the partner grid in a fixed device array
// of this file instead, so a call allocates nothing (no hipMalloc, no
// hipFree, no allocating library call): for callers that cannot allocate
// while they run, such as code under HIP graph capture or a serving loop.
//
// The array lives on every device the library runs on until the process
// ends.  Its device address is looked up once per device, on the first call
// there, with that device current; host code uses only that address (the
// array's name in host code is a host-side stand-in, not device memory).
// Every call on a device shares the device's array: calls that overlap in
// time on one device race and must be ordered by the caller (one stream, or
// events).  Nothing in the array needs to start at zero: every pass writes
// the whole grid before the next pass reads it.
#include <hip/hip_runtime.h>

#include <mutex>

#include "plan.hpp"
#include "stencil.h"

namespace {

constexpr int64_t kMaxCells = STENCIL_NOALLOC_MAX_CELLS;
constexpr int kMaxDevices = 64;

__device__ __align__(256) float scratch[kMaxCells];

std::mutex g_mu;
float *g_scratch[kMaxDevices] = {};

// Device address of this device's array (looked up once per device).
int scratch_address(int dev, float **ptr) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return star_set_error(STENCIL_EDEVICE, "hipGetSymbolAddress of the static scratch failed");
        }
        g_scratch[dev] = static_cast<float *>(p);
    }
    *ptr = g_scratch[dev];
    return STENCIL_OK;
}

}  // namespace

extern "C" int stencil_run_noalloc(stencil_plan_t plan, const float *in, float *out, int64_t steps,
                                   void *stream) {
    star_clear_error();
    int rc = run_check(plan, in, out, steps);
    if (rc != STENCIL_OK) return rc;
    if (plan->storage != STENCIL_F32)
        return star_set_error(STENCIL_EUNSUPPORTED,
                              "stencil_run_noalloc runs FP32 storage only (the precision form "
                              "keeps plan-owned buffers)");
    if (plan->ncells > kMaxCells)
        return star_set_error(STENCIL_EUNSUPPORTED,
                              "grid exceeds STENCIL_NOALLOC_MAX_CELLS cells (the static scratch)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return star_set_error(STENCIL_EDEVICE, "hipGetDevice failed");
    }
    float *part = nullptr;
    rc = scratch_address(dev, &part);
    if (rc != STENCIL_OK) return rc;
    const uintptr_t s0 = (uintptr_t)part, s1 = s0 + (uintptr_t)plan->ncells * sizeof(float);
    const uintptr_t bytes = (uintptr_t)plan->ncells * sizeof(float);
    if (((uintptr_t)in < s1 && s0 < (uintptr_t)in + bytes) ||
        ((uintptr_t)out < s1 && s0 < (uintptr_t)out + bytes))
        return star_set_error(STENCIL_EINVAL, "in/out overlap the static scratch");
    const hipStream_t st = (hipStream_t)stream;
    if (steps == 0) {
        if (hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, st) != hipSuccess) {
            (void)hipGetLastError();
            return star_set_error(STENCIL_EDEVICE, "hipMemcpyAsync failed");
        }
        return STENCIL_OK;
    }
    // the pass schedule of stencil_run (no host containers): floor(steps/K)
    // passes of K steps, then a tail pass; buffers alternate so that the
    // last pass writes `out`
    const int K = plan->K > 0 ? plan->K : 1;
    const int64_t full = steps / K, tail = steps % K;
    const int64_t np = full + (tail ? 1 : 0);
    const float *src = in;
    for (int64_t i = 0; i < np; ++i) {
        float *dst = ((np - 1 - i) % 2 == 0) ? out : part;
        const int k = i < full ? K : (int)tail;
        if (plan_launch_pass(plan, k, src, dst, st) != hipSuccess) {
            (void)hipGetLastError();
            return star_set_error(STENCIL_EDEVICE, "kernel launch failed");
        }
        src = dst;
    }
    return STENCIL_OK;
}
