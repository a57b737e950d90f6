// api.cpp -- the C ABI declared in include/stencil.h.
//
// Host side only: argument validation, coefficient copy, configuration
// choice, scratch ownership and the pass schedule (K fused steps per pass,
// ping-pong between the caller's output and the plan's scratch).  Every
// cell update runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "launch.hpp"
#include "plan.hpp"
#include "stencil.h"

using namespace star;

namespace {

thread_local std::string g_last_error;
std::atomic<uint64_t> g_plan_serial{0};

int fail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

int hip_fail(hipError_t e, const char *what) {
    return fail(STENCIL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool ranges_overlap(const void *a, const void *b, size_t bytes) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bytes && y < x + bytes;
}

}  // namespace

int star_set_error(int status, const char *msg) { return fail(status, "%s", msg); }
void star_clear_error() { g_last_error.clear(); }

int run_check(const stencil_plan_s *plan, const float *in, float *out, int64_t steps) {
    if (!plan) return fail(STENCIL_EINVAL, "plan is NULL");
    if (!in || !out) return fail(STENCIL_EINVAL, "in/out is NULL");
    if (steps < 0) return fail(STENCIL_EINVAL, "steps must be >= 0 (got %lld)", (long long)steps);
    if (((uintptr_t)in | (uintptr_t)out) & 3) return fail(STENCIL_EINVAL, "grids must be 4-byte aligned");
    const size_t bytes = (size_t)plan->ncells * sizeof(float);
    if (ranges_overlap(in, out, bytes)) return fail(STENCIL_EINVAL, "in and out overlap");
    if (ranges_overlap(in, plan->scratch, bytes) || ranges_overlap(out, plan->scratch, bytes))
        return fail(STENCIL_EINVAL, "in/out overlap the plan's scratch");
    if (plan->storage != STENCIL_F32 && ((uintptr_t)out & 15))
        return fail(STENCIL_EINVAL, "low-precision storage needs a 16-byte aligned out");
    return STENCIL_OK;
}

extern "C" {

const char *stencil_version(void) { return "mi355x-stencil 0.1 (gfx950)"; }

const char *stencil_status_string(int status) {
    switch (status) {
        case STENCIL_OK: return "ok";
        case STENCIL_EINVAL: return "invalid argument";
        case STENCIL_ENOMEM: return "out of memory";
        case STENCIL_EDEVICE: return "device error";
        case STENCIL_EUNSUPPORTED: return "unsupported";
        case STENCIL_EOVERFLOW: return "scale overflow";
        default: return "unknown status";
    }
}

const char *stencil_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"

namespace {

// Validates and builds a plan.  sym: the coefficients are shared per axis
// and distance (1 + ndim*radius values) instead of per point.
int plan_create(stencil_plan_t *plan, int ndim, const int64_t *dims, int radius,
                const float *coeffs, int ncoeffs, int boundary, int storage, int anchor_m,
                const char *tune, bool sym) {
    g_last_error.clear();
    if (!plan) return fail(STENCIL_EINVAL, "plan pointer is NULL");
    *plan = nullptr;
    if (ndim != 2 && ndim != 3) return fail(STENCIL_EINVAL, "ndim must be 2 or 3 (got %d)", ndim);
    if (!dims) return fail(STENCIL_EINVAL, "dims is NULL");
    if (radius < 1 || radius > 8) return fail(STENCIL_EINVAL, "radius must be 1..8 (got %d)", radius);
    if (!coeffs) return fail(STENCIL_EINVAL, "coeffs is NULL");
    const int npts = sym ? 1 + ndim * radius : 1 + 2 * ndim * radius;
    if (ncoeffs != npts)
        return fail(STENCIL_EINVAL, sym ? "ncoeffs must be 1+ndim*radius = %d (got %d)"
                                        : "ncoeffs must be 1+2*ndim*radius = %d (got %d)",
                    npts, ncoeffs);
    if (boundary != STENCIL_BOUNDARY_CLAMP && boundary != STENCIL_BOUNDARY_PADDED)
        return fail(STENCIL_EINVAL, "unknown boundary %d", boundary);
    if (storage < STENCIL_F32 || storage > STENCIL_BF16_SCALED)
        return fail(STENCIL_EINVAL, "unknown storage %d", storage);
    if (storage != STENCIL_F32 && anchor_m < 1)
        return fail(STENCIL_EINVAL, "anchor_m must be >= 1 for low-precision storage");
    if (boundary == STENCIL_BOUNDARY_PADDED && storage != STENCIL_F32)
        return fail(STENCIL_EUNSUPPORTED, "the padded-halo boundary is built for FP32 storage");
    if (sym && (boundary != STENCIL_BOUNDARY_CLAMP || storage != STENCIL_F32))
        return fail(STENCIL_EUNSUPPORTED, "shared coefficients are built for FP32 and the clamp boundary");
    if (sym && radius > 4)
        return fail(STENCIL_EUNSUPPORTED, "shared coefficients are built for radius 1..4");
    // padded-halo boundary: the arrays hold the interior inside a frame of
    // `radius` cells on every side
    const int pad = boundary == STENCIL_BOUNDARY_PADDED ? radius : 0;
    int64_t d[3] = {1, 1, 1};
    for (int a = 0; a < ndim; ++a) {
        if (dims[a] < 1) return fail(STENCIL_EINVAL, "dims[%d] = %lld < 1", a, (long long)dims[a]);
        if (dims[a] > (int64_t)1 << 30)
            return fail(STENCIL_EUNSUPPORTED, "dims[%d] = %lld exceeds 2^30", a, (long long)dims[a]);
        d[a] = dims[a] + 2 * pad;
    }
    const int64_t ncells = d[0] * d[1] * d[2];  // each factor <= 2^30: check before multiplying
    if ((double)d[0] * (double)d[1] * (double)d[2] * 4.0 > 9.0e18 || ncells > ((int64_t)1 << 40))
        return fail(STENCIL_EINVAL, "grid of %g cells overflows the byte size",
                    (double)d[0] * (double)d[1] * (double)d[2]);
    for (int k = 0; k < npts; ++k)
        if (!std::isfinite(coeffs[k])) return fail(STENCIL_EINVAL, "coefficient %d is not finite", k);

    auto *p = new (std::nothrow) stencil_plan_s();
    if (!p) return fail(STENCIL_ENOMEM, "host allocation failed");
    p->ndim = ndim;
    p->nx = d[0];
    p->ny = d[1];
    p->nz = d[2];
    p->ncells = ncells;
    p->radius = radius;
    p->npts = npts;
    std::memset(&p->cf, 0, sizeof p->cf);
    for (int k = 0; k < npts; ++k) p->cf.c[k] = coeffs[k];
    p->storage = storage;
    p->anchor_m = anchor_m;
    p->pad = pad;
    p->sym = sym ? 1 : 0;
    p->serial = ++g_plan_serial;
    // the configuration is validated before any device call, so a bad
    // request reports EINVAL even where no device is present
    hipError_t e = hipGetDevice(&p->device);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        p->device = -1;
    }
    int rc = plan_configure(p, tune);
    if (rc != STENCIL_OK) {
        delete p;
        return rc;
    }
    if (p->device < 0) {
        delete p;
        return hip_fail(e, "hipGetDevice");
    }
    e = hipMalloc(&p->scratch, (size_t)ncells * sizeof(float));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        delete p;
        return fail(STENCIL_ENOMEM, "hipMalloc of %lld-cell scratch failed: %s", (long long)ncells,
                    hipGetErrorString(e));
    }
    if (storage != STENCIL_F32) {
        rc = lowp_allocate(p);
        if (rc != STENCIL_OK) {
            stencil_plan_destroy(p);
            return rc;
        }
    }
    *plan = p;
    return STENCIL_OK;
}

}  // namespace

extern "C" {

int stencil_plan_ex(stencil_plan_t *plan, int ndim, const int64_t *dims, int radius,
                    const float *coeffs, int ncoeffs, int boundary, int storage, int anchor_m,
                    const char *tune) {
    return plan_create(plan, ndim, dims, radius, coeffs, ncoeffs, boundary, storage, anchor_m,
                       tune, false);
}

int stencil_plan_symmetric(stencil_plan_t *plan, int ndim, const int64_t *dims, int radius,
                           const float *axis_coeffs, int ncoeffs, int boundary, const char *tune) {
    return plan_create(plan, ndim, dims, radius, axis_coeffs, ncoeffs, boundary, STENCIL_F32, 0,
                       tune, true);
}

int stencil_coeffs_per_direction(int ndim, int radius, const float *per_direction, float *out) {
    g_last_error.clear();
    if (ndim != 2 && ndim != 3) return fail(STENCIL_EINVAL, "ndim must be 2 or 3 (got %d)", ndim);
    if (radius < 1 || radius > 8) return fail(STENCIL_EINVAL, "radius must be 1..8 (got %d)", radius);
    if (!per_direction || !out) return fail(STENCIL_EINVAL, "per_direction/out is NULL");
    out[0] = per_direction[0];
    for (int i = 1; i <= radius; ++i)
        for (int d = 0; d < 2 * ndim; ++d) out[1 + (i - 1) * 2 * ndim + d] = per_direction[1 + d];
    return STENCIL_OK;
}

int stencil_plan(stencil_plan_t *plan, int ndim, const int64_t *dims, int radius,
                 const float *coeffs, int ncoeffs, int boundary) {
    return stencil_plan_ex(plan, ndim, dims, radius, coeffs, ncoeffs, boundary, STENCIL_F32, 0,
                           nullptr);
}

void stencil_plan_destroy(stencil_plan_t plan) {
    if (!plan) return;
    if (plan->scratch) {
        // runs may still use the scratch on any stream of this device (the
        // plan does not record the caller's streams): wait for the device,
        // as hipFree would
        (void)hipDeviceSynchronize();
        (void)hipFree(plan->scratch);
    }
    plan_release_extra(plan);
    delete plan;
}

int stencil_plan_query(stencil_plan_t plan, int *K, int tile[3], int *vec,
                       double *bytes_per_cell_step) {
    if (!plan) return fail(STENCIL_EINVAL, "plan is NULL");
    if (K) *K = plan->K;
    if (tile) {
        tile[0] = plan->tile[0];
        tile[1] = plan->tile[1];
        tile[2] = plan->tile[2];
    }
    if (vec) *vec = plan->vec;
    if (bytes_per_cell_step) {
        if (plan->storage == STENCIL_F32) {
            *bytes_per_cell_step = 8.0 / plan->K;
        } else {
            const double m = plan->anchor_m;
            if (plan->storage == STENCIL_F16 || plan->storage == STENCIL_BF16) {
                // per window of m steps: G pass 8 B, encode 6 B, m-1 delta passes
                // of 6 B (read D and G, write D), re-anchor 10 B
                *bytes_per_cell_step = (6.0 * m + 18.0) / m;
            } else {
                // per window: tile maxima 4 B, encode 6 B, m-1 state passes of
                // 4 B, decode 6 B, FP32 anchor step 8 B
                *bytes_per_cell_step = (4.0 * m + 20.0) / m;
            }
        }
    }
    return STENCIL_OK;
}

int stencil_plan_describe(stencil_plan_t plan, char *buf, size_t len) {
    if (!plan) return fail(STENCIL_EINVAL, "plan is NULL");
    const std::string s = plan_describe(plan);
    if (buf && len > 0) {
        const size_t n = std::min(len - 1, s.size());
        std::memcpy(buf, s.data(), n);
        buf[n] = '\0';
    }
    return (int)s.size();
}

int stencil_run(stencil_plan_t plan, const float *in, float *out, int64_t steps, void *stream) {
    g_last_error.clear();
    const int rc = run_check(plan, in, out, steps);
    if (rc != STENCIL_OK) return rc;
    const hipError_t e = plan_enqueue(plan, in, out, steps, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, steps == 0 ? "hipMemcpyAsync" : "kernel launch");
    return STENCIL_OK;
}

}  // extern "C"
