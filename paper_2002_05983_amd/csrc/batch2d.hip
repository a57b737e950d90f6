// batch2d.hip -- persistent work-list kernel of the batched form, 2D grids.
//
// Compiled once per radius with -DSTAR_R=<1..8>.  Each wavefront takes one
// item (an x-strip and y-segment of one grid) at a time from the round's
// atomic counter and runs the same per-wavefront body as the single-grid
// kernel on it; wavefronts are independent (no barriers), so a workgroup's
// waves pull separately.
#include "batch.hpp"
#include "star2d_body.hpp"

#ifndef STAR_R
#error "compile with -DSTAR_R=<radius>"
#endif

namespace star {

namespace {

using s2d::prefetch_rows;
using s2d::star2d_body;

template <int R, int K, int D, bool ALIGNED>
__global__ __launch_bounds__(256) void star2d_batch(const BatchEntry *__restrict__ entries,
                                                    const BatchGrid *__restrict__ grids,
                                                    unsigned *counter, int nentries, int nitems) {
    const int lane = threadIdx.x & 63;
    for (;;) {
        unsigned got = 0;
        if (lane == 0) got = atomicAdd(counter, 1u);
        const int item = __builtin_amdgcn_readfirstlane((int)got);
        if (item >= nitems) break;
        const int ei = batch_find_entry(entries, nentries, item);
        const BatchEntry &en = entries[ei];
        const BatchGrid &g = grids[en.grid];
        const int t = item - en.item0;
        const Coefs cf = g.cf;
        star2d_body<R, K, D, ALIGNED>(en.src, en.dst, g.nx, g.ny, g.seg, t % en.ntx, t / en.ntx, cf);
    }
}

template <int K, bool AL>
const void *kernel_of() {
    return (const void *)star2d_batch<STAR_R, K, prefetch_rows<STAR_R, K>(), AL>;
}

template <int K>
const void *pick_al(bool aligned) {
    if constexpr (K > max_k2d(STAR_R)) {
        return nullptr;
    } else {
        return aligned ? kernel_of<K, true>() : kernel_of<K, false>();
    }
}

const void *pick(const BatchLaunchArgs &a) {
    switch (a.K) {
        case 1: return pick_al<1>(a.aligned);
        case 2: return pick_al<2>(a.aligned);
        case 3: return pick_al<3>(a.aligned);
        case 4: return pick_al<4>(a.aligned);
        case 5: return pick_al<5>(a.aligned);
        case 6: return pick_al<6>(a.aligned);
        case 7: return pick_al<7>(a.aligned);
        case 8: return pick_al<8>(a.aligned);
        case 9: return pick_al<9>(a.aligned);
        case 10: return pick_al<10>(a.aligned);
        default: return nullptr;
    }
}

}  // namespace

#define STAR_CAT2(a, b) a##b
#define STAR_CAT(a, b) STAR_CAT2(a, b)

int STAR_CAT(batch2d_occupancy_r, STAR_R)(const BatchLaunchArgs &a) {
    const void *k = pick(a);
    if (!k) return 0;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 256, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return nb;
}

hipError_t STAR_CAT(launch_batch2d_r, STAR_R)(const BatchLaunchArgs &a, hipStream_t s) {
    const void *k = pick(a);
    if (!k || a.blocks < 1 || a.nentries < 1 || a.nitems < 1) return hipErrorInvalidValue;
    void *args[] = {(void *)&a.entries, (void *)&a.grids, (void *)&a.counter,
                    (void *)&a.nentries, (void *)&a.nitems};
    return hipLaunchKernel(k, dim3((unsigned)a.blocks), dim3(256), args, 0, s);
}

}  // namespace star
