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

// pad > 0 (padded-halo boundary, Sec. IV.B): the grid is the padded array;
// cells of its frame of `pad` cells keep their values.  SYM: shared
// coefficients (c_C, then c_x,i, c_y,i[, c_z,i] for i = 1..R), one FMA per
// axis and distance with the rounded sum of the pair.
template <int NDIM, int R, bool SYM>
__global__ __launch_bounds__(256) void star_naive(const float *__restrict__ src,
                                                  float *__restrict__ dst, int nx, int ny,
                                                  int nz, int64_t ncells, int pad, Coefs cf) {
    const int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (p >= ncells) return;
    const int x = (int)(p % nx);
    const int y = (int)((p / nx) % ny);
    const int z = (int)(p / ((int64_t)nx * ny));
    auto at = [&](int xx, int yy, int zz) -> float {
        return src[(int64_t)xx + (int64_t)nx * ((int64_t)yy + (int64_t)ny * zz)];
    };
    if (pad > 0 && (x < pad || x >= nx - pad || y < pad || y >= ny - pad ||
                    (NDIM == 3 && (z < pad || z >= nz - pad)))) {
        dst[p] = at(x, y, z);
        return;
    }
    float acc = cf.c[0] * at(x, y, z);
#pragma unroll
    for (int i = 1; i <= R; ++i) {
        const float w = at(clampi(x - i, nx), y, z), e = at(clampi(x + i, nx), y, z);
        const float s = at(x, clampi(y - i, ny), z), n = at(x, clampi(y + i, ny), z);
        if constexpr (SYM) {
            acc = __builtin_fmaf(cf.c[1 + (i - 1) * NDIM], w + e, acc);
            acc = __builtin_fmaf(cf.c[2 + (i - 1) * NDIM], s + n, acc);
            if constexpr (NDIM == 3) {
                const float b = at(x, y, clampi(z - i, nz)), a = at(x, y, clampi(z + i, nz));
                acc = __builtin_fmaf(cf.c[3 + (i - 1) * NDIM], b + a, acc);
            }
        } else {
            acc = __builtin_fmaf(cf.c[coef_index<NDIM>(kW, i)], w, acc);
            acc = __builtin_fmaf(cf.c[coef_index<NDIM>(kE, i)], e, acc);
            acc = __builtin_fmaf(cf.c[coef_index<NDIM>(kS, i)], s, acc);
            acc = __builtin_fmaf(cf.c[coef_index<NDIM>(kN, i)], n, acc);
            if constexpr (NDIM == 3) {
                acc = __builtin_fmaf(cf.c[coef_index<NDIM>(kB, i)], at(x, y, clampi(z - i, nz)), acc);
                acc = __builtin_fmaf(cf.c[coef_index<NDIM>(kA, i)], at(x, y, clampi(z + i, nz)), acc);
            }
        }
    }
    dst[p] = acc;
}

template <int NDIM, int R>
static hipError_t launch_one(const float *src, float *dst, int nx, int ny, int nz,
                             const Coefs &cf, hipStream_t stream, int pad, bool sym) {
    const int64_t n = (int64_t)nx * ny * nz;
    const int64_t blocks = (n + 255) / 256;
    // the dispatch's work-item count is 32-bit
    if (blocks * 256 > (int64_t)0xFFFFFFFF) return hipErrorInvalidValue;
    if (sym)
        hipLaunchKernelGGL((star_naive<NDIM, R, true>), dim3((unsigned)blocks), dim3(256), 0, stream,
                           src, dst, nx, ny, nz, n, pad, cf);
    else
        hipLaunchKernelGGL((star_naive<NDIM, R, false>), dim3((unsigned)blocks), dim3(256), 0, stream,
                           src, dst, nx, ny, nz, n, pad, cf);
    return hipGetLastError();
}

hipError_t launch_naive(int ndim, int R, const float *src, float *dst, int nx, int ny, int nz,
                        const Coefs &cf, hipStream_t stream, int pad, bool sym) {
    if (ndim == 2) nz = 1;
#define CASE(ND, RR) \
    if (ndim == ND && R == RR) return launch_one<ND, RR>(src, dst, nx, ny, nz, cf, stream, pad, sym);
    CASE(2, 1) CASE(2, 2) CASE(2, 3) CASE(2, 4) CASE(2, 5) CASE(2, 6) CASE(2, 7) CASE(2, 8)
    CASE(3, 1) CASE(3, 2) CASE(3, 3) CASE(3, 4) CASE(3, 5) CASE(3, 6) CASE(3, 7) CASE(3, 8)
#undef CASE
    return hipErrorInvalidValue;
}

}  // namespace star
