// star3d_rows.hip -- single-grid launch of the LDS-free 3D single-step pass
// (method in star3d_rows.hpp).
//
// Compiled once per radius with -DSTAR_R=<1..8>.
#include "star3d_rows.hpp"

#ifndef STAR_R
#error "compile with -DSTAR_R=<radius>"
#endif

namespace star {

namespace {

using s3r::prefetch_rows3;
using s3r::star3d_rows_body;

// Four wavefronts per workgroup, each independent.  Up to radius 4
// wavefront w takes strip w % nstrips of row block (w / nstrips) % nyb and
// z-segment w / (nstrips * nyb); above radius 4 the row block runs fastest
// (row block w % nyb of strip (w / nyb) % nstrips).  Either way consecutive
// wavefronts (one workgroup, one CU; and, through the XCD-aware block
// order, one L2) hold neighbouring rows at the same planes, so the
// y-neighbour rows they load from each other are cache hits; strip-first
// also keeps the halo columns of adjacent strips together (measured on
// 512^3, row block first: R = 1, 2 -11 and -7 %, R = 3, 4 -1 %, R = 5, 6,
// 8 +3, +3, +4 %).  WPE: waves per SIMD the register budget is sized for.
// LPR: lanes per grid row (64, or 16: four rows of a 64-column strip per
// wavefront, for narrow grids).
template <int R, int RPL, bool NBP, bool AL, int WPE, bool SYM, int LPR>
__global__ __launch_bounds__(256, WPE) void star3d_rows(const float *__restrict__ src,
                                                        float *__restrict__ dst, int nx, int ny,
                                                        int nz, int nstrips, int nyb, int lz,
                                                        int nwaves, int pad, Coefs cf) {
    const int wave = xcd_logical_block(blockIdx.x, gridDim.x) * 4 +
                     __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wave >= nwaves) return;
    constexpr bool YFIRST = R > 4;
    const int yb = YFIRST ? wave % nyb : (wave / nstrips) % nyb;
    const int strip = YFIRST ? (wave / nyb) % nstrips : wave % nstrips;
    const int zseg = wave / (nstrips * nyb);
    constexpr int D = prefetch_rows3<R, RPL>();
    constexpr int RPW = RPL * (64 / LPR);  // grid rows per wavefront
    if (AL && (strip + 1) * LPR * 4 > nx)
        star3d_rows_body<R, RPL, D, NBP, AL, true, SYM, LPR>(src, dst, nx, ny, nz, strip, yb * RPW,
                                                             zseg * lz, lz, cf, pad);
    else
        star3d_rows_body<R, RPL, D, NBP, AL, false, SYM, LPR>(src, dst, nx, ny, nz, strip, yb * RPW,
                                                              zseg * lz, lz, cf, pad);
}

template <int RPL, bool NBP, bool AL, bool SYM = false, int LPR = 64>
hipError_t launch_rows(const Star3DArgs &a, hipStream_t stream) {
    constexpr int SW = LPR * 4, RPW = RPL * (64 / LPR);
    const int nstrips = (a.nx + SW - 1) / SW;
    const int nyb = (a.ny + RPW - 1) / RPW;
    const int nseg = (a.nz + a.lz - 1) / a.lz;
    const int64_t nwaves = (int64_t)nstrips * nyb * nseg;
    if (nwaves > ((int64_t)1 << 30)) return hipErrorInvalidValue;
    if ((int64_t)a.nx * a.ny * (int64_t)sizeof(float) >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    // 4 waves per SIMD (128 VGPRs) where the ring and neighbour rows fit,
    // else 2 (256 VGPRs): two rows per wavefront, radius >= 5, and the
    // heavier radius-4 forms
    constexpr int R = STAR_R;
    constexpr int WPE = (RPL == 1 && (R <= 3 || (R == 4 && AL && !NBP))) ? 4 : 2;
    const unsigned blocks = (unsigned)((nwaves + 3) / 4);
    hipLaunchKernelGGL((star3d_rows<STAR_R, RPL, NBP, AL, WPE, SYM, LPR>), dim3(blocks), dim3(256), 0,
                       stream, a.src, a.dst, a.nx, a.ny, a.nz, nstrips, nyb, a.lz, (int)nwaves,
                       a.pad, a.cf);
    return hipGetLastError();
}

}  // namespace

#define STAR_CAT2(a, b) a##b
#define STAR_CAT(a, b) STAR_CAT2(a, b)

hipError_t STAR_CAT(launch_star3d_rows_r, STAR_R)(const Star3DArgs &a, hipStream_t stream) {
    if (a.lz < 1 || a.nx < 1 || a.ny < 1 || a.nz < 1 || a.K != 1) return hipErrorInvalidValue;
    if (a.lpr == 16) {
        // 16 lanes per row: one row per group, no prefetch, per-point coefficients
        if constexpr (STAR_R <= 4) {
            if (a.rows != 1 || a.nbp || a.sym) return hipErrorInvalidValue;
            return a.aligned ? launch_rows<1, false, true, false, 16>(a, stream)
                             : launch_rows<1, false, false, false, 16>(a, stream);
        }
        return hipErrorInvalidValue;
    }
    if (a.lpr != 64) return hipErrorInvalidValue;
    if (a.sym) {
        // shared coefficients: one row per wavefront, radius <= 4
        if constexpr (STAR_R <= 4) {
            if (!a.aligned) return launch_rows<1, false, false, true>(a, stream);
            return a.nbp ? launch_rows<1, true, true, true>(a, stream)
                         : launch_rows<1, false, true, true>(a, stream);
        }
        return hipErrorInvalidValue;
    }
    if (!a.aligned) {
        if (a.rows != 1 || a.nbp) return hipErrorInvalidValue;  // built for one row, no prefetch
        return launch_rows<1, false, false>(a, stream);
    }
    if (a.rows == 1) return a.nbp ? launch_rows<1, true, true>(a, stream) : launch_rows<1, false, true>(a, stream);
    if (a.rows == 2) {
        if constexpr (STAR_R <= 4)
            return a.nbp ? launch_rows<2, true, true>(a, stream) : launch_rows<2, false, true>(a, stream);
        else  // two rows per wavefront above radius 4: no neighbour prefetch (registers)
            return a.nbp ? hipErrorInvalidValue : launch_rows<2, false, true>(a, stream);
    }
    if constexpr (STAR_R <= 4) {
        // four rows per wavefront: 2R neighbour rows per 4 output rows
        if (a.rows == 4 && !a.nbp) return launch_rows<4, false, true>(a, stream);
    }
    return hipErrorInvalidValue;
}

}  // namespace star
