// batch.hpp -- work lists of the batched form (internal).
//
// A batch runs many independent grids.  Grids are grouped into classes
// (dimension, radius, alignment, size); every class has one kernel
// configuration and runs as a chain of pass rounds.  One pass round of a
// class is one launch of a persistent work-list kernel: its workgroups
// (2D: its wavefronts) take items -- one x-strip/y-segment (2D) or one
// xy-tile/z-segment (3D) of one grid -- from an atomic counter until the
// round's list is exhausted.  An item is the same unit of work as one
// wavefront (2D) or workgroup (3D) of the single-grid kernels, done by the
// same device code, so a grid's result does not depend on how it is run.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace star {

// A grid as the work-list kernels see it.
struct BatchGrid {
    Coefs cf;
    int nx, ny, nz;
    int seg;  // output rows (2D) or planes (3D) per segment
};

// One grid's share of one launch: items [item0, next entry's item0).
// Item t of the grid is strip t % ntx, then (3D) tile row band
// (t / ntx) % nty, then segment t / (ntx * nty) (2D: nty = 1).
struct BatchEntry {
    const float *src;
    float *dst;
    int grid;  // index into the grid table
    int item0;
    int ntx;   // x-strips
    int nty;   // 3D: tile row bands
    int hx;    // 3D: x halo columns per side
    int tx;    // 3D: output columns per strip
};

struct BatchLaunchArgs {
    const BatchEntry *entries;  // sorted by item0; entries[0].item0 == 0
    const BatchGrid *grids;
    unsigned *counter;          // must read 0 when the launch starts
    int nentries;
    int nitems;
    int blocks;                 // persistent workgroups to launch
    int K;                      // steps fused in this round
    bool aligned;               // every grid: nx % 4 == 0, src/dst 16-byte aligned
    // 3D configuration
    int vec, wl, nw;
};

hipError_t launch_batch2d_r1(const BatchLaunchArgs &a, hipStream_t s);
hipError_t launch_batch2d_r2(const BatchLaunchArgs &a, hipStream_t s);
hipError_t launch_batch2d_r3(const BatchLaunchArgs &a, hipStream_t s);
hipError_t launch_batch2d_r4(const BatchLaunchArgs &a, hipStream_t s);
hipError_t launch_batch3d_r1(const BatchLaunchArgs &a, hipStream_t s);
hipError_t launch_batch3d_r2(const BatchLaunchArgs &a, hipStream_t s);
hipError_t launch_batch3d_r3(const BatchLaunchArgs &a, hipStream_t s);
hipError_t launch_batch3d_r4(const BatchLaunchArgs &a, hipStream_t s);
// Resident workgroups per CU of the kernel that `a` selects (K, aligned and,
// for 3D, vec/wl/nw); the 3D query also sets the kernel's dynamic-LDS limit,
// so it must run before the kernel's first launch and outside of stream
// capture.  0 = configuration not built.
int batch2d_occupancy_r1(const BatchLaunchArgs &a);
int batch2d_occupancy_r2(const BatchLaunchArgs &a);
int batch2d_occupancy_r3(const BatchLaunchArgs &a);
int batch2d_occupancy_r4(const BatchLaunchArgs &a);
int batch3d_occupancy_r1(const BatchLaunchArgs &a);
int batch3d_occupancy_r2(const BatchLaunchArgs &a);
int batch3d_occupancy_r3(const BatchLaunchArgs &a);
int batch3d_occupancy_r4(const BatchLaunchArgs &a);

// Index of the entry holding `item`: the last entry whose item0 <= item.
// Wave-level (every lane of the wavefront calls it with the same item).
__device__ __forceinline__ int batch_find_entry(const BatchEntry *__restrict__ e, int n, int item) {
    const int lane = threadIdx.x & 63;
    int idx = 0;
    for (int b = 0; b < n; b += 64) {
        const int l = b + lane;
        const bool le = l < n && e[l].item0 <= item;
        const int c = __builtin_popcountll(__ballot(le));
        idx = c > 0 ? b + c - 1 : idx;
        if (c < 64) break;
    }
    return __builtin_amdgcn_readfirstlane(idx);
}

}  // namespace star
