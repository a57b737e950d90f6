// star2d.hip -- single-grid launch of the 2D star stencil (method in star2d_body.hpp).
//
// Compiled once per radius with -DSTAR_R=<1..8>.
#include "star2d_body.hpp"

#ifndef STAR_R
#error "compile with -DSTAR_R=<radius>"
#endif

namespace star {

namespace {

using s2d::prefetch_rows;
using s2d::star2d_body;

template <int R, int K, int D, bool ALIGNED, bool SYM>
__global__ __launch_bounds__(256) void star2d_stream(const float *__restrict__ src,
                                                     float *__restrict__ dst, int nx, int ny,
                                                     int ly, int nstrips, int nwaves, int pad,
                                                     Coefs cf) {
    // Everything that does not depend on the lane is wave-uniform; the
    // readfirstlane makes the compiler keep it in scalar registers and turn
    // the per-row conditions into scalar branches.
    const int wave = xcd_logical_block(blockIdx.x, gridDim.x) * 4 +
                     __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nwaves) return;
    const int strip = wave % nstrips, seg = wave / nstrips;
    if (s2d::star2d_interior<R, K>(nx, ny, ly, strip, seg, pad))
        star2d_body<R, K, D, ALIGNED, false, SYM>(src, dst, nx, ny, ly, strip, seg, cf);
    else
        star2d_body<R, K, D, ALIGNED, true, SYM>(src, dst, nx, ny, ly, strip, seg, cf, pad);
}

template <int K, bool AL, bool SYM>
hipError_t launch_k(const Star2DArgs &a, hipStream_t stream) {
    constexpr int TX = star2d_tile_x(K, STAR_R);
    const int nstrips = (a.nx + TX - 1) / TX;
    const int nsegs = (a.ny + a.ly - 1) / a.ly;
    const int64_t nwaves = (int64_t)nstrips * nsegs;
    if (nwaves > (int64_t)1 << 30) return hipErrorInvalidValue;
    // one row is one buffer descriptor: its byte size and masked offsets stay below 2^31
    if ((int64_t)a.nx * (int64_t)sizeof(float) >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    const unsigned blocks = (unsigned)((nwaves + 3) / 4);
    hipLaunchKernelGGL((star2d_stream<STAR_R, K, prefetch_rows<STAR_R, K>(), AL, SYM>), dim3(blocks),
                       dim3(256), 0, stream, a.src, a.dst, a.nx, a.ny, a.ly, nstrips, (int)nwaves,
                       a.pad, a.cf);
    return hipGetLastError();
}

template <int K>
hipError_t launch_al(const Star2DArgs &a, hipStream_t stream) {
    if constexpr (K > max_k2d(STAR_R)) {
        return hipErrorInvalidValue;
    } else {
        if (a.sym) {
            if constexpr (STAR_R <= 4 && K <= kMaxKSym2D)
                return a.aligned ? launch_k<K, true, true>(a, stream) : launch_k<K, false, true>(a, stream);
            return hipErrorInvalidValue;
        }
        return a.aligned ? launch_k<K, true, false>(a, stream) : launch_k<K, false, false>(a, stream);
    }
}

}  // namespace

#define STAR_CAT2(a, b) a##b
#define STAR_CAT(a, b) STAR_CAT2(a, b)

hipError_t STAR_CAT(launch_star2d_r, STAR_R)(const Star2DArgs &a, hipStream_t stream) {
    if (a.ly < 1 || a.nx < 1 || a.ny < 1) return hipErrorInvalidValue;
    switch (a.K) {
        case 1: return launch_al<1>(a, stream);
        case 2: return launch_al<2>(a, stream);
        case 3: return launch_al<3>(a, stream);
        case 4: return launch_al<4>(a, stream);
        case 5: return launch_al<5>(a, stream);
        case 6: return launch_al<6>(a, stream);
        case 7: return launch_al<7>(a, stream);
        case 8: return launch_al<8>(a, stream);
        case 9: return launch_al<9>(a, stream);
        case 10: return launch_al<10>(a, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace star
