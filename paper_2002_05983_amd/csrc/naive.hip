// naive.hip -- one thread per cell, one time step per launch.
//
// The plain form of Eq. (1) (Sec. IV.A) with the clamp boundary of Sec. III.B:
// each thread reads its 1 + 2*ndim*R clamped neighbours straight from memory
// and writes one cell.  It is the library's reference variant ("naive"): the
// blocked kernels must reproduce it bit for bit, since all variants evaluate
// the same FP32 operation sequence.
#include "common.hpp"
#include "launch.hpp"

namespace star {

template <int NDIM, int R>
__global__ __launch_bounds__(256) void star_naive(const float *__restrict__ src,
                                                  float *__restrict__ dst, int nx, int ny,
                                                  int nz, int64_t ncells, Coefs cf) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= ncells) return;
    const int x = (int)(p % nx);
    const int y = (int)((p / nx) % ny);
    const int z = (int)(p / ((int64_t)nx * ny));
    auto at = [&](int xx, int yy, int zz) -> float {
        return src[(int64_t)xx + (int64_t)nx * ((int64_t)yy + (int64_t)ny * zz)];
    };
    float acc = cf.c[0] * at(x, y, z);
#pragma unroll
    for (int i = 1; i <= R; ++i) {
        acc = __builtin_fmaf(cf.c[coef_index<NDIM>(kW, i)], at(clampi(x - i, nx), y, z), acc);
        acc = __builtin_fmaf(cf.c[coef_index<NDIM>(kE, i)], at(clampi(x + i, nx), y, z), acc);
        acc = __builtin_fmaf(cf.c[coef_index<NDIM>(kS, i)], at(x, clampi(y - i, ny), z), acc);
        acc = __builtin_fmaf(cf.c[coef_index<NDIM>(kN, i)], at(x, clampi(y + i, ny), z), acc);
        if constexpr (NDIM == 3) {
            acc = __builtin_fmaf(cf.c[coef_index<NDIM>(kB, i)], at(x, y, clampi(z - i, nz)), acc);
            acc = __builtin_fmaf(cf.c[coef_index<NDIM>(kA, i)], at(x, y, clampi(z + i, nz)), acc);
        }
    }
    dst[p] = acc;
}

template <int NDIM, int R>
static hipError_t launch_one(const float *src, float *dst, int nx, int ny, int nz,
                             const Coefs &cf, hipStream_t stream) {
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t blocks = (n + 255) / 256;
    // the dispatch's work-item count is 32-bit
    if (blocks * 256 > (int64_t)0xFFFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL((star_naive<NDIM, R>), dim3((unsigned)blocks), dim3(256), 0, stream, src,
                       dst, nx, ny, nz, n, cf);
    return hipGetLastError();
}

hipError_t launch_naive(int ndim, int R, const float *src, float *dst, int nx, int ny, int nz,
                        const Coefs &cf, hipStream_t stream) {
    if (ndim == 2) nz = 1;
#define CASE(ND, RR) \
    if (ndim == ND && R == RR) return launch_one<ND, RR>(src, dst, nx, ny, nz, cf, stream);
    CASE(2, 1) CASE(2, 2) CASE(2, 3) CASE(2, 4) CASE(2, 5) CASE(2, 6) CASE(2, 7) CASE(2, 8)
    CASE(3, 1) CASE(3, 2) CASE(3, 3) CASE(3, 4) CASE(3, 5) CASE(3, 6) CASE(3, 7) CASE(3, 8)
#undef CASE
    return hipErrorInvalidValue;
}

}  // namespace star
