// common.hpp -- shared device helpers of the gfx950 star-stencil kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

// Lambdas inside kernels are forced inline: the register queues they touch
// must stay in registers, which needs every access at a compile-time index.
#define STAR_INLINE __attribute__((always_inline))

namespace star {

// Largest point count: a radius-8 3D star (1 + 2*3*8).
constexpr int kMaxPoints = 49;

// Per-point coefficients, passed by value in the kernel argument segment so
// that every coefficient is a scalar register operand of the FMA chain.
// Order: c_C, then for i = 1..R the directions W, E, S, N (, B, A).
struct Coefs {
    float c[kMaxPoints];
};

// Index of neighbour (direction slot d, distance i) for an ndim-D star.
template <int NDIM>
__host__ __device__ constexpr int coef_index(int d, int i) {
    return 1 + (i - 1) * 2 * NDIM + d;
}
enum : int { kW = 0, kE = 1, kS = 2, kN = 3, kB = 4, kA = 5 };

constexpr int gcd_i(int a, int b) { return b == 0 ? a : gcd_i(b, a % b); }

template <int I, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

__device__ __forceinline__ int clampi(int v, int n) { return v < 0 ? 0 : (v >= n ? n - 1 : v); }

// Whole-wavefront lane shifts (DPP wave_shr:1 / wave_shl:1, full-rate VALU
// moves).  The lane with no source (lane 0, resp. lane 63) gets `edge`:
// callers pass the lane's own outermost cell, which is the clamped value
// when a row starts (ends) at that lane.
__device__ __forceinline__ float from_lower_lane(float v, float edge) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, v), 0x138,
                                                                 0xf, 0xf, false));
}
__device__ __forceinline__ float from_upper_lane(float v, float edge) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, v), 0x130,
                                                                 0xf, 0xf, false));
}
// The same shifts within each row of L lanes: L = 64 is the whole-wavefront
// shift above; L = 16 shifts inside every 16-lane DPP row (row_shr:1 /
// row_shl:1), and the first (last) lane of each row gets `edge`.
template <int L>
__device__ __forceinline__ float from_lower_lane_in(float v, float edge) {
    static_assert(L == 64 || L == 16, "rows of 64 or 16 lanes");
    if constexpr (L == 64) return from_lower_lane(v, edge);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, v), 0x111,
                                                                 0xf, 0xf, false));
}
template <int L>
__device__ __forceinline__ float from_upper_lane_in(float v, float edge) {
    static_assert(L == 64 || L == 16, "rows of 64 or 16 lanes");
    if constexpr (L == 64) return from_upper_lane(v, edge);
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, edge),
                                                                 __builtin_bit_cast(int, v), 0x101,
                                                                 0xf, 0xf, false));
}
// The same shifts where the lane with no source may receive anything (zero).
__device__ __forceinline__ float from_lower_lane_or_zero(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xf,
                                                              0xf, true));
}
__device__ __forceinline__ float from_upper_lane_or_zero(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xf,
                                                              0xf, true));
}
// Fused wave shift: a += c * (v of the lane below / above) as one
// v_fmac_f32 with the wave shift on its first operand, in place of a
// v_mov_b32_dpp and a v_fmac_f32 (the compiler fuses DPP moves into adds
// and multiplies but not into FMAs).  The lane with no source reads 0.
// Each result is the same correctly rounded fma(c, v_shifted, a).  c must
// be in a VGPR (vgpr_copy).  The s_nop 1 gives the two wait states a DPP
// read needs after a VALU write of its source register, which the compiler
// does not insert for inline assembly; within a block no instruction
// writes a shifted source.
#define STAR_FSH(dir, a, v, c) "v_fmac_f32_dpp %" #a ", %" #v ", %" #c " " dir \
    " row_mask:0xf bank_mask:0xf bound_ctrl:1\n\t"
// Both sides of one distance I in one block (4 cells per lane): a[e] +=
// cw * (vw[e] of the lane below) for the first min(I, 4) cells, then
// a[e] += ce * (ve[k] of the lane above) for the last min(I, 4) cells
// (k = e - (4 - min(I, 4))): every cell still takes its W term before its
// E term, and the block needs the wait states once.
template <int I>
__device__ __forceinline__ void fma_shifted_we(float (&a)[4], float cw, const float *vw, float ce,
                                               const float *ve) {
    static_assert(I >= 1, "distance >= 1");
    if constexpr (I == 1) {
        asm("s_nop 1\n\t" STAR_FSH("wave_shr:1", 0, 2, 4) STAR_FSH("wave_shl:1", 1, 3, 5)
            : "+v"(a[0]), "+v"(a[3]) : "v"(vw[0]), "v"(ve[0]), "v"(cw), "v"(ce));
    } else if constexpr (I == 2) {
        asm("s_nop 1\n\t" STAR_FSH("wave_shr:1", 0, 4, 8) STAR_FSH("wave_shr:1", 1, 5, 8)
                STAR_FSH("wave_shl:1", 2, 6, 9) STAR_FSH("wave_shl:1", 3, 7, 9)
            : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3])
            : "v"(vw[0]), "v"(vw[1]), "v"(ve[0]), "v"(ve[1]), "v"(cw), "v"(ce));
    } else if constexpr (I == 3) {
        asm("s_nop 1\n\t" STAR_FSH("wave_shr:1", 0, 4, 10) STAR_FSH("wave_shr:1", 1, 5, 10)
                STAR_FSH("wave_shr:1", 2, 6, 10) STAR_FSH("wave_shl:1", 1, 7, 11)
                STAR_FSH("wave_shl:1", 2, 8, 11) STAR_FSH("wave_shl:1", 3, 9, 11)
            : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3])
            : "v"(vw[0]), "v"(vw[1]), "v"(vw[2]), "v"(ve[0]), "v"(ve[1]), "v"(ve[2]), "v"(cw),
              "v"(ce));
    } else {
        asm("s_nop 1\n\t" STAR_FSH("wave_shr:1", 0, 4, 12) STAR_FSH("wave_shr:1", 1, 5, 12)
                STAR_FSH("wave_shr:1", 2, 6, 12) STAR_FSH("wave_shr:1", 3, 7, 12)
                STAR_FSH("wave_shl:1", 0, 8, 13) STAR_FSH("wave_shl:1", 1, 9, 13)
                STAR_FSH("wave_shl:1", 2, 10, 13) STAR_FSH("wave_shl:1", 3, 11, 13)
            : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3])
            : "v"(vw[0]), "v"(vw[1]), "v"(vw[2]), "v"(vw[3]), "v"(ve[0]), "v"(ve[1]), "v"(ve[2]),
              "v"(ve[3]), "v"(cw), "v"(ce));
    }
}
#undef STAR_FSH
// W and E coefficients of distances 1..R held in VGPRs, for the FMAs that
// take their operand from the adjacent lane through fma_shifted.
template <int R>
struct XCoefV {
    float w[R + 1], e[R + 1];
};

// A wave-uniform value copied into a VGPR (an operand that must be a VGPR).
__device__ __forceinline__ float vgpr_copy(float s) {
    float v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(s));
    return v;
}

// Value of v in lane `lane` (wave-uniform lane index), broadcast to all lanes.
__device__ __forceinline__ float lane_value(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// Raw buffer resources (gfx9 layout: stride 0, byte-range checked).  An
// access at a byte offset >= the resource's size is dropped by the hardware
// (a store writes nothing, a load returns 0), which masks lanes without a
// branch.  Sizes must stay below 2^31 bytes so kOutOfRange is out of range.
typedef int v4i __attribute__((ext_vector_type(4)));
constexpr int kRsrcWord3 = 0x00020000;
constexpr int kOutOfRange = (int)0x80000000u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, bytes, kRsrcWord3);
}
// Byte offset `off` (< 2^31) when `ok`, else an out-of-range offset: the top
// bit is or-ed in, so the store stays one unconditional instruction.
__device__ __forceinline__ int masked_offset(int off, bool ok) {
    return (int)((unsigned)off | ((unsigned)(!ok) << 31));
}
// Cache-policy bits of a store (gfx950): 2 marks it non-temporal, for
// outputs a pass never reads again, so that they do not push rows other
// wavefronts are about to read out of L2.
constexpr int kStoreNT = 2;
template <int AUX = 0>
__device__ __forceinline__ void buffer_store4(__amdgpu_buffer_rsrc_t r, int off, float a, float b,
                                              float c, float d) {
    const v4i v = {__builtin_bit_cast(int, a), __builtin_bit_cast(int, b),
                   __builtin_bit_cast(int, c), __builtin_bit_cast(int, d)};
    __builtin_amdgcn_raw_buffer_store_b128(v, r, off, 0, AUX);
}
template <int AUX = 0>
__device__ __forceinline__ void buffer_store1(__amdgpu_buffer_rsrc_t r, int off, float a) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(int, a), r, off, 0, AUX);
}

// Workgroups are handed to the 8 XCDs of the chip round-robin by block id.
// Renumber them so that each XCD works on one contiguous range of logical
// blocks (neighbouring tiles, whose halos overlap, then share an L2).
__device__ __forceinline__ int xcd_logical_block(int b, int nblocks) {
    const int q = nblocks >> 3, r = nblocks & 7, x = b & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

}  // namespace star
