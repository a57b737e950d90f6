// lowp.hpp -- low-precision storage of the precision form (internal).
//
// A stored value is a 16-bit code q (FP16 or BF16) and the power-of-two
// scale 2^e of its 64^3 storage tile: value = q * 2^e.  Decoding and scaling
// are exact; encoding rounds v * 2^-e to the nearest code, ties to even.
// The tile exponent is e = ceil(log2 B) - 14 for a bound B >= max|v| of the
// tile (e = 0 when B = 0), so |q| <= 2^14, two binades below FP16's largest
// finite value.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace star {

enum : int { kCodecF16 = 1, kCodecBF16 = 2 };
constexpr int kTileShift = 6;  // 64^3 storage tiles
constexpr int kHeadroomBits = 14;

template <int CODEC>
__device__ __forceinline__ float decode_code(uint32_t q16, int e) {
    float f;
    if constexpr (CODEC == kCodecF16) {
        f = (float)__builtin_bit_cast(_Float16, (uint16_t)q16);
    } else {
        f = __builtin_bit_cast(float, q16 << 16);
    }
    return __builtin_amdgcn_ldexpf(f, e);
}

template <int CODEC>
__device__ __forceinline__ uint32_t encode_code(float v, int e) {
    const float s = __builtin_amdgcn_ldexpf(v, -e);
    if constexpr (CODEC == kCodecF16) {
        return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)s);
    } else {
        const uint32_t b = __builtin_bit_cast(uint32_t, s);
        return (b + 0x7FFFu + ((b >> 16) & 1u)) >> 16;  // round to nearest, ties to even
    }
}

// Tile exponent for a bound B >= 0 (computed in double on both the host
// model and the device).
__host__ __device__ inline int tile_exponent(double B) {
    if (!(B > 0.0)) return 0;
    int k = 0;
    const double m = frexp(B, &k);  // B = m * 2^k, m in [0.5, 1)
    const int c = (m == 0.5) ? k - 1 : k;  // ceil(log2 B)
    return c - kHeadroomBits;
}

struct LowpArgs {
    // D pass: codes in / G codes / codes out; G pass: f32 in / f32 out
    const uint16_t *d_in;
    const int *e_in;
    const uint16_t *g;
    const int *e_g;
    uint16_t *d_out;
    const int *e_out;
    const float *a_in;      // G pass input (FP32 anchor)
    float *g_out;           // G pass output (FP32 staging)
    unsigned *max_out;      // per-tile max |value| before rounding (float bits)
    int nx, ny, nz;
    int nw, wl, lz;
    int tnx, tny, tnz;      // storage tiles per axis
    Coefs cf;
};

// mode 0: G pass (FP32 in/out); mode kCodecF16/kCodecBF16: delta pass
// D' = encode(S decode(D) + decode(G)); mode kScaledPass + codec: state pass
// Q' = encode(S decode(Q)) (no G term).
constexpr int kScaledPass = 2;
hipError_t launch_lowp3d_r1(const LowpArgs &a, int mode, hipStream_t s);
hipError_t launch_lowp3d_r2(const LowpArgs &a, int mode, hipStream_t s);
hipError_t launch_lowp3d_r3(const LowpArgs &a, int mode, hipStream_t s);
hipError_t launch_lowp3d_r4(const LowpArgs &a, int mode, hipStream_t s);

// Elementwise and per-tile helpers (lowp_util.hip).
hipError_t lowp_fill_u32(unsigned *p, int64_t n, unsigned v, hipStream_t s);
hipError_t lowp_exponents_from_max(const unsigned *maxv, int ntiles, int *e, hipStream_t s);
hipError_t lowp_exponents_from_bound(const unsigned *max_d, const unsigned *max_g, double s1,
                                     int tnx, int tny, int tnz, int *e, hipStream_t s);
// G16 = encode(G32) with per-tile exponents e_g.
hipError_t lowp_encode(int codec, const float *g32, const int *e_g, uint16_t *g16, int nx, int ny,
                       int nz, int tnx, int tny, hipStream_t s);
// max |x| per tile of an FP32 field (into maxv, which must start at 0)
hipError_t lowp_tile_max(const float *x32, unsigned *maxv, int nx, int ny, int nz, int tnx, int tny,
                         hipStream_t s);
// out = a + decode(d), or decode(d) when a is null  (out may alias a)
hipError_t lowp_add_decoded(int codec, const float *a, const uint16_t *d, const int *e_d,
                            float *out, int nx, int ny, int nz, int tnx, int tny, hipStream_t s);

}  // namespace star
