// star3d.hip -- single-grid launch of the 3D star stencil (method in star3d_body.hpp).
//
// Compiled once per radius with -DSTAR_R=<1..4>.
#include "star3d_body.hpp"

#ifndef STAR_R
#error "compile with -DSTAR_R=<radius>"
#endif

namespace star {

namespace {

using s3d::prefetch3;
using s3d::star3d_body;

template <int R, int K, int VEC, int WL, int D, bool ALIGNED, bool PAIR>
__global__ __launch_bounds__(1024) void star3d_stream(const float *__restrict__ src,
                                                      float *__restrict__ dst, int nx, int ny,
                                                      int nz, int hx, int tx, int ntx, int nty,
                                                      int lz, int pad, Coefs cf) {
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int strip = lb % ntx, ytile = (lb / ntx) % nty, zseg = lb / (ntx * nty);
    const int nt = (blockDim.x >> 6) * (64 / WL);
    if (s3d::star3d_interior<R, K, VEC, WL>(nx, ny, nz, hx, tx, strip, ytile, zseg, lz, nt, pad))
        star3d_body<R, K, VEC, WL, D, ALIGNED, false, PAIR>(src, dst, nx, ny, nz, hx, tx, strip,
                                                            ytile, zseg, lz, cf);
    else
        star3d_body<R, K, VEC, WL, D, ALIGNED, true, PAIR>(src, dst, nx, ny, nz, hx, tx, strip,
                                                           ytile, zseg, lz, cf, pad);
}

template <int K, int VEC, int WL, bool AL, bool PAIR = false>
hipError_t launch_k3(const Star3DArgs &a, hipStream_t stream) {
    constexpr int R = STAR_R;
    constexpr int W = WL * VEC;
    const int nw = a.nw;
    const int nt = nw * (64 / WL);
    const int ty = nt - 2 * K * R;
    if (ty < 1 || nw > 16 || nw < 1) return hipErrorInvalidValue;
    int hx = 0, tx = a.nx, ntx = 1;
    if (a.nx > W || WL != 64) {
        hx = (K * R + VEC - 1) / VEC * VEC;
        tx = W - 2 * hx;
        ntx = (a.nx + tx - 1) / tx;
    }
    const int nty = (a.ny + ty - 1) / ty;
    const int nseg = (a.nz + a.lz - 1) / a.lz;
    const int64_t blocks = (int64_t)ntx * nty * nseg;
    if (blocks > ((int64_t)1 << 30)) return hipErrorInvalidValue;
    if ((int64_t)a.nx * a.ny * (int64_t)sizeof(float) >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    // two LDS buffers per stage, four for the paired form
    const size_t lds = (size_t)K * (PAIR ? 4 : 2) * nt * W * sizeof(float);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    auto kern = star3d_stream<R, K, VEC, WL, prefetch3<STAR_R, K, VEC, WL>(), AL, PAIR>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(nw * 64), lds, stream, a.src, a.dst,
                       a.nx, a.ny, a.nz, hx, tx, ntx, nty, a.lz, a.pad, a.cf);
    return hipGetLastError();
}

template <int K>
hipError_t launch_kv(const Star3DArgs &a, hipStream_t stream) {
    if constexpr (K > max_k3d(STAR_R)) {
        return hipErrorInvalidValue;
    } else {
        if constexpr (K == 1) {
            if (a.pair && a.vec == 4 && a.wl == 64)
                return a.aligned ? launch_k3<K, 4, 64, true, true>(a, stream)
                                 : launch_k3<K, 4, 64, false, true>(a, stream);
            if (a.pair && a.vec == 4 && a.wl == 32)
                return a.aligned ? launch_k3<K, 4, 32, true, true>(a, stream)
                                 : launch_k3<K, 4, 32, false, true>(a, stream);
        }
        if (a.pair) return hipErrorInvalidValue;  // single-step, 4 cells per lane only
        if (a.vec == 4 && a.wl == 64)
            return a.aligned ? launch_k3<K, 4, 64, true>(a, stream) : launch_k3<K, 4, 64, false>(a, stream);
        if (a.vec == 4 && a.wl == 32)
            return a.aligned ? launch_k3<K, 4, 32, true>(a, stream) : launch_k3<K, 4, 32, false>(a, stream);
        if constexpr (K == 1 && STAR_R <= 2) {
            // a 512-column row per wavefront: only the aligned single-step
            // pass of radius <= 2 fits in the register budget
            if (a.vec == 8 && a.wl == 64 && a.aligned) return launch_k3<K, 8, 64, true>(a, stream);
        }
        return hipErrorInvalidValue;
    }
}

}  // namespace

#define STAR_CAT2(a, b) a##b
#define STAR_CAT(a, b) STAR_CAT2(a, b)

hipError_t STAR_CAT(launch_star3d_r, STAR_R)(const Star3DArgs &a, hipStream_t stream) {
    if (a.lz < 1 || a.nx < 1 || a.ny < 1 || a.nz < 1) return hipErrorInvalidValue;
    if (a.sym) return hipErrorInvalidValue;  // shared coefficients run the row layout
    switch (a.K) {
        case 1: return launch_kv<1>(a, stream);
        case 2: return launch_kv<2>(a, stream);
        case 3: return launch_kv<3>(a, stream);
        case 4: return launch_kv<4>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace star
