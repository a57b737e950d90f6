// batch3d.hip -- persistent work-list kernel of the batched form, 3D grids.
//
// Compiled once per radius with -DSTAR_R=<1..4>.  A workgroup takes one
// item (an xy-tile and z-segment of one grid) at a time from the round's
// atomic counter -- thread 0 draws it, a barrier publishes it -- and runs
// the same per-workgroup body as the single-grid kernel on it.
#include "batch.hpp"
#include "star3d_body.hpp"

#ifndef STAR_R
#error "compile with -DSTAR_R=<radius>"
#endif

namespace star {

namespace {

using s3d::prefetch3;
using s3d::star3d_body;

template <int R, int K, int VEC, int WL, int D, bool ALIGNED>
__global__ __launch_bounds__(1024) void star3d_batch(const BatchEntry *__restrict__ entries,
                                                     const BatchGrid *__restrict__ grids,
                                                     unsigned *counter, int nentries, int nitems,
                                                     int slot_off) {
    extern __shared__ float lds[];
    // the item slot sits after the body's LDS rows
    unsigned *slot = reinterpret_cast<unsigned *>(lds + slot_off);
    for (;;) {
        __syncthreads();  // every wave is done with the previous item and its slot
        if (threadIdx.x == 0) *slot = atomicAdd(counter, 1u);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane((int)*slot);
        if (item >= nitems) break;
        const int ei = batch_find_entry(entries, nentries, item);
        const BatchEntry &en = entries[ei];
        const BatchGrid &g = grids[en.grid];
        const int t = item - en.item0;
        const Coefs cf = g.cf;
        star3d_body<R, K, VEC, WL, D, ALIGNED>(en.src, en.dst, g.nx, g.ny, g.nz, en.hx, en.tx,
                                               t % en.ntx, (t / en.ntx) % en.nty,
                                               t / (en.ntx * en.nty), g.seg, cf);
    }
}

template <int K, int VEC, int WL, bool AL>
const void *kernel_of() {
    return (const void *)star3d_batch<STAR_R, K, VEC, WL, prefetch3<STAR_R, K, VEC, WL>(), AL>;
}

template <int K>
const void *pick_k(const BatchLaunchArgs &a) {
    if constexpr (K > max_k3d(STAR_R)) {
        return nullptr;
    } else {
        if (a.vec == 4 && a.wl == 64) return a.aligned ? kernel_of<K, 4, 64, true>() : kernel_of<K, 4, 64, false>();
        if (a.vec == 4 && a.wl == 32) return a.aligned ? kernel_of<K, 4, 32, true>() : kernel_of<K, 4, 32, false>();
        if constexpr (K == 1 && STAR_R <= 2) {
            if (a.vec == 8 && a.wl == 64 && a.aligned) return kernel_of<K, 8, 64, true>();
        }
        return nullptr;
    }
}

const void *pick(const BatchLaunchArgs &a) {
    if (a.nw < 1 || a.nw > 16) return nullptr;
    if (a.nw * (64 / (a.wl > 0 ? a.wl : 64)) - 2 * a.K * STAR_R < 1) return nullptr;
    switch (a.K) {
        case 1: return pick_k<1>(a);
        case 2: return pick_k<2>(a);
        case 3: return pick_k<3>(a);
        case 4: return pick_k<4>(a);
        default: return nullptr;
    }
}

// Floats of the body's LDS rows: K stages x 2 buffers x tile rows x row.
int body_floats(const BatchLaunchArgs &a) {
    return a.K * 2 * a.nw * (64 / a.wl) * a.wl * a.vec;
}

}  // namespace

#define STAR_CAT2(a, b) a##b
#define STAR_CAT(a, b) STAR_CAT2(a, b)

int STAR_CAT(batch3d_occupancy_r, STAR_R)(const BatchLaunchArgs &a) {
    const void *k = pick(a);
    if (!k) return 0;
    const size_t lds = (size_t)body_floats(a) * sizeof(float) + 16;
    if (lds > 160 * 1024) return 0;
    // the limit covers every class that shares this kernel, whatever its tile
    if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, a.nw * 64, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

hipError_t STAR_CAT(launch_batch3d_r, STAR_R)(const BatchLaunchArgs &a, hipStream_t s) {
    const void *k = pick(a);
    if (!k || a.blocks < 1 || a.nentries < 1 || a.nitems < 1) return hipErrorInvalidValue;
    int slot_off = body_floats(a);
    const size_t lds = (size_t)slot_off * sizeof(float) + 16;
    void *args[] = {(void *)&a.entries, (void *)&a.grids,    (void *)&a.counter,
                    (void *)&a.nentries, (void *)&a.nitems, (void *)&slot_off};
    return hipLaunchKernel(k, dim3((unsigned)a.blocks), dim3(a.nw * 64), args, lds, s);
}

}  // namespace star
