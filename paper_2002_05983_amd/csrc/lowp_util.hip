// lowp_util.hip -- elementwise and per-tile kernels of the precision form.
//
// Storage tiles are 64^3 cells; tile t = (z/64 * tny + y/64) * tnx + x/64.
// The elementwise kernels give each wavefront one 256-column chunk of one
// 64-row band of one plane (each lane 4 columns, looping over the rows), so
// the 16 lanes of one storage tile reduce their maxima with cross-lane
// shuffles and a single atomic per tile per wavefront.  All grids here have
// nx % 4 == 0.
#include <algorithm>

#include "lowp.hpp"

namespace star {

namespace {

__global__ __launch_bounds__(256) void fill_u32(unsigned *p, int64_t n, unsigned v) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        p[i] = v;
}

__global__ __launch_bounds__(256) void exp_from_max(const unsigned *maxv, int ntiles, int *e) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t < ntiles) e[t] = tile_exponent((double)__uint_as_float(maxv[t]));
}

__global__ __launch_bounds__(256) void exp_from_bound(const unsigned *max_d, const unsigned *max_g,
                                                      double s1, int tnx, int tny, int tnz, int *e) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= tnx * tny * tnz) return;
    const int tx = t % tnx, ty = (t / tnx) % tny, tz = t / (tnx * tny);
    float m = 0.0f;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx) {
                const int x = tx + dx, y = ty + dy, z = tz + dz;
                if (x < 0 || y < 0 || z < 0 || x >= tnx || y >= tny || z >= tnz) continue;
                m = fmaxf(m, __uint_as_float(max_d[(z * tny + y) * tnx + x]));
            }
    e[t] = tile_exponent(s1 * (double)m + (double)__uint_as_float(max_g[t]));
}

struct Chunk {
    int x0, y0, y1, z;
    bool live;
};
__device__ __forceinline__ Chunk chunk_of(int nx, int ny, int nz, int wave) {
    const int ncx = (nx + 255) / 256, nby = (ny + 63) / 64;
    Chunk c;
    c.z = wave / (ncx * nby);
    const int rem = wave % (ncx * nby);
    c.y0 = (rem / ncx) * 64;
    c.y1 = min(c.y0 + 64, ny);
    c.x0 = (rem % ncx) * 256;
    c.live = c.z < nz;
    return c;
}

template <int CODEC>
__global__ __launch_bounds__(256) void encode_k(const float *__restrict__ g32, const int *__restrict__ e_g,
                                                uint16_t *__restrict__ g16, int nx, int ny, int nz,
                                                int tnx, int tny) {
    const int lane = threadIdx.x & 63;
    const Chunk c = chunk_of(nx, ny, nz, blockIdx.x * 4 + (threadIdx.x >> 6));
    if (!c.live) return;
    const int x = c.x0 + lane * 4;
    const bool in = x < nx;
    const int t = ((c.z >> kTileShift) * tny + (c.y0 >> kTileShift)) * tnx + (min(x, nx - 4) >> kTileShift);
    const int e = e_g[t];
    if (in) {
        for (int y = c.y0; y < c.y1; ++y) {
            const size_t off = ((size_t)c.z * ny + y) * nx + x;
            const float4 v = *reinterpret_cast<const float4 *>(g32 + off);
            const uint32_t q0 = encode_code<CODEC>(v.x, e), q1 = encode_code<CODEC>(v.y, e);
            const uint32_t q2 = encode_code<CODEC>(v.z, e), q3 = encode_code<CODEC>(v.w, e);
            *reinterpret_cast<uint2 *>(g16 + off) = make_uint2(q0 | (q1 << 16), q2 | (q3 << 16));
        }
    }
}

__global__ __launch_bounds__(256) void tile_max_k(const float *__restrict__ x32, unsigned *__restrict__ maxv,
                                                  int nx, int ny, int nz, int tnx, int tny) {
    const int lane = threadIdx.x & 63;
    const Chunk c = chunk_of(nx, ny, nz, blockIdx.x * 4 + (threadIdx.x >> 6));
    if (!c.live) return;
    const int x = c.x0 + lane * 4;
    const bool in = x < nx;
    const int t = ((c.z >> kTileShift) * tny + (c.y0 >> kTileShift)) * tnx + (min(x, nx - 4) >> kTileShift);
    float m = 0.0f;
    if (in) {
        for (int y = c.y0; y < c.y1; ++y) {
            const float4 v = *reinterpret_cast<const float4 *>(x32 + ((size_t)c.z * ny + y) * nx + x);
            m = fmaxf(m, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
        }
    }
    for (int s = 8; s >= 1; s >>= 1) m = fmaxf(m, __shfl_xor(m, s, 16));
    if ((lane & 15) == 0 && in) atomicMax(maxv + t, __float_as_uint(m));
}

// out = a + decode(d), or decode(d) when a is null
template <int CODEC>
__global__ __launch_bounds__(256) void add_decoded_k(const float *a, const uint16_t *__restrict__ d,
                                                     const int *__restrict__ e_d, float *out, int nx,
                                                     int ny, int nz, int tnx, int tny) {
    const int lane = threadIdx.x & 63;
    const Chunk c = chunk_of(nx, ny, nz, blockIdx.x * 4 + (threadIdx.x >> 6));
    if (!c.live) return;
    const int x = c.x0 + lane * 4;
    if (x >= nx) return;
    const int e = e_d[((c.z >> kTileShift) * tny + (c.y0 >> kTileShift)) * tnx + (x >> kTileShift)];
    for (int y = c.y0; y < c.y1; ++y) {
        const size_t off = ((size_t)c.z * ny + y) * nx + x;
        const float4 v = a ? *reinterpret_cast<const float4 *>(a + off) : make_float4(0.f, 0.f, 0.f, 0.f);
        const uint2 q = *reinterpret_cast<const uint2 *>(d + off);
        *reinterpret_cast<float4 *>(out + off) =
            make_float4(v.x + decode_code<CODEC>(q.x & 0xFFFFu, e), v.y + decode_code<CODEC>(q.x >> 16, e),
                        v.z + decode_code<CODEC>(q.y & 0xFFFFu, e), v.w + decode_code<CODEC>(q.y >> 16, e));
    }
}

unsigned chunk_blocks(int nx, int ny, int nz) {
    const int64_t waves = (int64_t)((nx + 255) / 256) * ((ny + 63) / 64) * nz;
    return (unsigned)((waves + 3) / 4);
}

}  // namespace

hipError_t lowp_fill_u32(unsigned *p, int64_t n, unsigned v, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_u32, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t lowp_exponents_from_max(const unsigned *maxv, int ntiles, int *e, hipStream_t s) {
    hipLaunchKernelGGL(exp_from_max, dim3((ntiles + 255) / 256), dim3(256), 0, s, maxv, ntiles, e);
    return hipGetLastError();
}

hipError_t lowp_exponents_from_bound(const unsigned *max_d, const unsigned *max_g, double s1,
                                     int tnx, int tny, int tnz, int *e, hipStream_t s) {
    const int n = tnx * tny * tnz;
    hipLaunchKernelGGL(exp_from_bound, dim3((n + 255) / 256), dim3(256), 0, s, max_d, max_g, s1,
                       tnx, tny, tnz, e);
    return hipGetLastError();
}

hipError_t lowp_tile_max(const float *x32, unsigned *maxv, int nx, int ny, int nz, int tnx, int tny,
                         hipStream_t s) {
    hipLaunchKernelGGL(tile_max_k, dim3(chunk_blocks(nx, ny, nz)), dim3(256), 0, s, x32, maxv, nx, ny,
                       nz, tnx, tny);
    return hipGetLastError();
}

hipError_t lowp_encode(int codec, const float *g32, const int *e_g, uint16_t *g16, int nx, int ny,
                       int nz, int tnx, int tny, hipStream_t s) {
    const unsigned blocks = chunk_blocks(nx, ny, nz);
    if (codec == kCodecF16)
        hipLaunchKernelGGL(encode_k<kCodecF16>, dim3(blocks), dim3(256), 0, s, g32, e_g, g16, nx, ny,
                           nz, tnx, tny);
    else
        hipLaunchKernelGGL(encode_k<kCodecBF16>, dim3(blocks), dim3(256), 0, s, g32, e_g, g16, nx, ny,
                           nz, tnx, tny);
    return hipGetLastError();
}

hipError_t lowp_add_decoded(int codec, const float *a, const uint16_t *d, const int *e_d, float *out,
                            int nx, int ny, int nz, int tnx, int tny, hipStream_t s) {
    const unsigned blocks = chunk_blocks(nx, ny, nz);
    if (codec == kCodecF16)
        hipLaunchKernelGGL(add_decoded_k<kCodecF16>, dim3(blocks), dim3(256), 0, s, a, d, e_d, out,
                           nx, ny, nz, tnx, tny);
    else
        hipLaunchKernelGGL(add_decoded_k<kCodecBF16>, dim3(blocks), dim3(256), 0, s, a, d, e_d, out,
                           nx, ny, nz, tnx, tny);
    return hipGetLastError();
}

}  // namespace star
