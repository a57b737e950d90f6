// launch.hpp -- host-side launchers of the kernel families (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace star {

// One step per launch, one thread per cell (reference variant).  pad > 0:
// padded-halo frame of that width kept fixed; sym: shared coefficients per
// axis and distance.
hipError_t launch_naive(int ndim, int R, const float *src, float *dst, int nx, int ny, int nz,
                        const Coefs &cf, hipStream_t stream, int pad = 0, bool sym = false);

// 2D x-strip / y-stream kernel fusing K steps per pass.
struct Star2DArgs {
    const float *src;
    float *dst;
    int nx, ny;
    int K;        // steps fused in this pass (1..max_k2d(R))
    int ly;       // output rows per y-segment
    bool aligned; // nx % 4 == 0 and both grids 16-byte aligned
    int pad = 0;  // padded-halo boundary: width of the fixed frame (0 = clamp)
    bool sym = false;  // shared coefficients per axis and distance (R <= 4, K <= 4)
    Coefs cf;
};
constexpr int kMaxK2D = 10;
// Shared coefficients (one per axis and distance) are built into the 2D
// streaming kernel for R <= 4 and K <= kMaxKSym2D fused steps.
constexpr int kMaxKSym2D = 4;
// Largest K built per radius: K*R <= 16 keeps the unrolled queue code and
// its registers in budget (K = 10, 8, 5, 4, 3, 2, 2, 2 for R = 1..8; at
// R = 1, K = 12 needs 172 VGPRs, two wavefronts per SIMD, and is slower
// than K = 10: 4045 against 4670 GCell/s on 16384^2).
constexpr int max_k2d(int R) { return 16 / R < kMaxK2D ? 16 / R : kMaxK2D; }
constexpr int kVec2D = 4;
// Output columns of one strip: a wavefront spans 64*4 columns, minus the
// overlapped halo of roundup(K*R, 4) columns per side (Eq. (2) analogue).
constexpr int star2d_halo(int K, int R) { return (K * R + kVec2D - 1) / kVec2D * kVec2D; }
constexpr int star2d_tile_x(int K, int R) { return 64 * kVec2D - 2 * star2d_halo(K, R); }

hipError_t launch_star2d_r1(const Star2DArgs &a, hipStream_t stream);
hipError_t launch_star2d_r2(const Star2DArgs &a, hipStream_t stream);
hipError_t launch_star2d_r3(const Star2DArgs &a, hipStream_t stream);
hipError_t launch_star2d_r4(const Star2DArgs &a, hipStream_t stream);
hipError_t launch_star2d_r5(const Star2DArgs &a, hipStream_t stream);
hipError_t launch_star2d_r6(const Star2DArgs &a, hipStream_t stream);
hipError_t launch_star2d_r7(const Star2DArgs &a, hipStream_t stream);
hipError_t launch_star2d_r8(const Star2DArgs &a, hipStream_t stream);

// 3D xy-tile / z-stream kernel fusing K steps per pass.
struct Star3DArgs {
    const float *src;
    float *dst;
    int nx, ny, nz;
    int K;        // steps fused in this pass
    int vec;      // cells per lane along x: 4 or 8
    int wl;       // lanes per tile row: 64 or 32 (two rows per wavefront)
    int nw;       // wavefronts per workgroup; tile rows = nw*64/wl incl. 2*K*R halo rows
    int lz;       // output planes per z-segment
    bool pair;    // two planes per barrier (k = 1, vec = 4)
    bool aligned; // nx % 4 == 0 and both grids 16-byte aligned
    int rows = 0; // LDS-free single-step layout: grid rows per wavefront (1, 2), 0 = xy tiles
    bool nbp = false;  // rows layout: neighbour rows loaded one plane ahead
    int lpr = 64;      // rows layout: lanes per grid row, 64 or 16 (narrow grids, R <= 4)
    int pad = 0;  // padded-halo boundary: width of the fixed frame (0 = clamp)
    bool sym = false;  // shared coefficients per axis and distance (row layout, R <= 4)
    Coefs cf;
};
// Largest K built per radius: the tile keeps >= 8 output rows of 16 for
// R = 1 and every build stays within 128 VGPRs without spilling.
constexpr int max_k3d(int R) { return R == 1 ? 4 : R <= 3 ? 3 : R <= 6 ? 2 : 1; }
// Widest row: 512 columns (vec 8) for aligned single-step passes of R <= 2.
constexpr bool vec8_ok(int R, int K, bool aligned) { return K == 1 && R <= 2 && aligned; }

hipError_t launch_star3d_r1(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_r2(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_r3(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_r4(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_r5(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_r6(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_r7(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_r8(const Star3DArgs &a, hipStream_t stream);

// LDS-free 3D single-step pass: whole 256-column rows per wavefront, z
// streamed, y-neighbour rows loaded from the caches (star3d_rows.hpp).
hipError_t launch_star3d_rows_r1(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_rows_r2(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_rows_r3(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_rows_r4(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_rows_r5(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_rows_r6(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_rows_r7(const Star3DArgs &a, hipStream_t stream);
hipError_t launch_star3d_rows_r8(const Star3DArgs &a, hipStream_t stream);

}  // namespace star
