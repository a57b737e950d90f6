// reduce.hip -- FP64 error-norm and conservation-sum reductions.
//
// max|x - ref|, max|ref| and sum(x), accumulated in FP64 on the GPU: the
// normwise relative L-infinity error of an FP32 (or low-precision) result
// against an FP64 reference, and the sum of the field (conserved when the
// coefficients sum to 1 and no cell is clamped away; used as a diagnostic).
// The grid size and the reduction tree are fixed, so the sum is bitwise
// reproducible from run to run.  The maxima propagate NaN: a NaN (or an
// infinity, whose difference from a finite reference is infinite and from
// an infinite one NaN) anywhere in x or ref shows in the result instead of
// being skipped, as a plain fmax would.
#include <hip/hip_runtime.h>

#include <mutex>

#include "stencil.h"

namespace star {

namespace {

constexpr int kBlocks = 1024;
constexpr int kThreads = 256;

// max(a, b) that returns NaN when either operand is NaN.
__device__ __forceinline__ double max_nan(double a, double b) { return (a > b || a != a) ? a : b; }

__global__ __launch_bounds__(kThreads) void reduce_partials(const float *__restrict__ x,
                                                            const double *__restrict__ ref,
                                                            int64_t n, double *__restrict__ part) {
    double md = 0.0, mr = 0.0, sm = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kThreads;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) {
        const double xv = (double)x[i];
        sm += xv;
        if (ref) {
            const double rv = ref[i];
            md = max_nan(md, fabs(xv - rv));
            mr = max_nan(mr, fabs(rv));
        }
    }
    __shared__ double s[3][kThreads];
    s[0][threadIdx.x] = md;
    s[1][threadIdx.x] = mr;
    s[2][threadIdx.x] = sm;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] = max_nan(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = max_nan(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] = s[2][threadIdx.x] + s[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = s[0][0];
        part[3 * blockIdx.x + 1] = s[1][0];
        part[3 * blockIdx.x + 2] = s[2][0];
    }
}

__global__ __launch_bounds__(kThreads) void reduce_final(const double *__restrict__ part, int np,
                                                         double *__restrict__ out) {
    __shared__ double s[3][kThreads];
    double md = 0.0, mr = 0.0, sm = 0.0;
    for (int i = threadIdx.x; i < np; i += kThreads) {
        md = max_nan(md, part[3 * i + 0]);
        mr = max_nan(mr, part[3 * i + 1]);
        sm += part[3 * i + 2];
    }
    s[0][threadIdx.x] = md;
    s[1][threadIdx.x] = mr;
    s[2][threadIdx.x] = sm;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s[0][threadIdx.x] = max_nan(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = max_nan(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] = s[2][threadIdx.x] + s[2][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = s[0][0];
        out[1] = s[1][0];
        out[2] = s[2][0];
    }
}

// Per-device workspace: kBlocks partial triples plus the final triple.
std::mutex g_mu;
double *g_work[64] = {};

}  // namespace

}  // namespace star

int star_set_error(int status, const char *msg);

extern "C" int stencil_reduce_f64(const float *x, const double *ref, int64_t n, double out[3],
                                  void *stream) {
    using namespace star;
    if (!x || !out) return star_set_error(STENCIL_EINVAL, "x/out is NULL");
    if (n < 1) return star_set_error(STENCIL_EINVAL, "n must be >= 1");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64)
        return star_set_error(STENCIL_EDEVICE, "hipGetDevice failed");
    double *work = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_work[dev]) {
            if (hipMalloc(&g_work[dev], sizeof(double) * 3 * (kBlocks + 1)) != hipSuccess) {
                (void)hipGetLastError();
                g_work[dev] = nullptr;
                return star_set_error(STENCIL_ENOMEM, "reduction workspace allocation failed");
            }
        }
        work = g_work[dev];
    }
    hipStream_t st = (hipStream_t)stream;
    const int64_t want = (n + kThreads - 1) / kThreads;
    const int blocks = (int)(want < kBlocks ? want : kBlocks);
    hipLaunchKernelGGL(reduce_partials, dim3(blocks), dim3(kThreads), 0, st, x, ref, n, work);
    hipLaunchKernelGGL(reduce_final, dim3(1), dim3(kThreads), 0, st, work, blocks,
                       work + 3 * kBlocks);
    if (hipGetLastError() != hipSuccess)
        return star_set_error(STENCIL_EDEVICE, "reduction launch failed");
    double host[3];
    if (hipMemcpyAsync(host, work + 3 * kBlocks, sizeof host, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
        return star_set_error(STENCIL_EDEVICE, "reduction copy-back failed");
    out[0] = host[0];
    out[1] = host[1];
    out[2] = host[2];
    return STENCIL_OK;
}
