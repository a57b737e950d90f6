// lowp3d.hip -- single-step 3D passes of the precision form.
//
// Compiled once per radius with -DSTAR_R=<1..4>.
//
// The precision form keeps an FP32 anchor A and a low-precision delta D
// (F = A + D); because one step S of Eq. (1) is linear (the clamp only
// copies cells), D evolves as D <- S D + G with G = S A - A fixed between
// anchors.  Two passes are built here on the same 2.5D scheme as the FP32
// kernel (xy tile with LDS rows, z streamed through a register window of
// 2R+1 planes, x-neighbours by DPP, one barrier per plane):
//   mode 0  G pass:  G32 = S A - A  (FP32 in, FP32 out), per-tile max|G|
//   mode 1  D pass:  D' = encode(S decode(D) + decode(G)) with FP16 codes
//   mode 2  D pass:  the same with BF16 codes
//   mode 3/4 state pass of the scaled-state form: Q' = encode(S decode(Q))
//           with FP16/BF16 codes (the D pass without its G term)
// Every value of the window is FP32; each cell is c_C*f_C followed by one
// FMA per neighbour in coefficient order, then (D pass) one FP32 add of G.
// Codes are decoded when their plane enters the window; the exponents of a
// lane's storage tile are re-read only when the z-tile changes.  The output
// tile exponents were fixed before the pass from a bound on |D'|, and the
// pass records max|value| (before rounding to a code) per output tile for
// the next bound.
#include "lowp.hpp"

#ifndef STAR_R
#error "compile with -DSTAR_R=<radius>"
#endif

namespace star {

namespace {

constexpr int VEC = 4;
typedef int v2i __attribute__((ext_vector_type(2)));

// one LDS row of a tile: WL lanes x 4 floats, lane-major
__device__ __forceinline__ void lds_write_row4(float *row, int lr, const float (&v)[VEC]) {
    *reinterpret_cast<float4 *>(row + lr * 4) = make_float4(v[0], v[1], v[2], v[3]);
}
__device__ __forceinline__ void lds_read_row4(const float *row, int lr, float (&v)[VEC]) {
    const float4 t = *reinterpret_cast<const float4 *>(row + lr * 4);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
}

// Raw rings (input codes or floats, and G codes) of NR planes: NR - 1
// planes in flight ahead of the one entering the window.
template <int R>
constexpr int default_ring() {
    constexpr int P = 2 * R + 1;
    return (P == 9) ? 3 : (P < 4 ? P : 4);
}

template <int R, int WL, int MODE, bool HAS_G, int NR>
__global__ __launch_bounds__(1024) void lowp3d_step(LowpArgs a, int hx, int tx, int ntx, int nty) {
    constexpr int P = 2 * R + 1;   // window planes
    constexpr int U = P * NR / gcd_i(P, NR);  // planes per unrolled loop trip
    constexpr int RPW = 64 / WL;
    constexpr int W = WL * VEC;
    constexpr bool FP32_IN = MODE == 0;
    extern __shared__ float lds[];  // [2][NT][W]

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int lane = threadIdx.x & 63;
    const int lr = lane % WL;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nt = (blockDim.x >> 6) * RPW;
    const int ty = nt - 2 * R;
    const int lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int strip = lb % ntx;
    const int ytile = (lb / ntx) % nty;
    const int zseg = lb / (ntx * nty);
    const int ty0 = ytile * ty;
    const int trow = w * RPW + lane / WL;
    const int y = ty0 - R + trow;
    const int yc = clampi(y, ny);
    const bool load_only = (w * RPW + RPW - 1 < R) || (w * RPW >= nt - R);
    const int xs = strip * tx - hx;
    const int col0 = xs + lr * VEC;
    const int z0 = zseg * a.lz;
    const int z1 = min(z0 + a.lz, nz);
    const int zstart = z0 - R;
    const int niter = (z1 - z0) + 2 * R;
    const int zlast = zstart + niter - 1;
    const bool left_edge = xs < 0;
    const bool right_edge = xs + W > nx;
    const int out_lo = max(xs + hx, 0);
    const int out_hi = min(xs + hx + tx, nx);
    const bool row_out = y >= ty0 && y < ty0 + ty && y < ny;
    const size_t plane = (size_t)nx * (size_t)ny;
    const int cl = min(max(col0, 0), nx - VEC);  // clamped vector column (16-byte aligned)
    // storage tile of this lane's column and row; z varies
    const int tile_xy = (yc >> kTileShift) * a.tnx + (cl >> kTileShift);
    const int tile_zstride = a.tnx * a.tny;

    auto lds_row = [&](int b, int r) STAR_INLINE -> float * {
        return lds + ((size_t)(b * nt + r)) * W;
    };
    auto tile_row = [&](int yy) STAR_INLINE -> int {
        const int r = clampi(yy, ny) - (ty0 - R);
        return r < 0 ? 0 : (r >= nt ? nt - 1 : r);
    };
    auto row_value = [&](float v, int l) STAR_INLINE -> float {
        float b = lane_value(v, l);
#pragma unroll
        for (int k = 1; k < RPW; ++k) b = (lane / WL == k) ? lane_value(v, k * WL + l) : b;
        return b;
    };
    auto xfix = [&](float (&v)[VEC]) STAR_INLINE {
        if (left_edge) {
            const int l0 = (-xs) / VEC;
            const float b = row_value(v[0], l0);
            if (lr < l0) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[e] = b;
            }
        }
        if (right_edge) {
            const int off = nx - 1 - xs;
            const int lrr = off / VEC, er = off % VEC;
            float t = v[0];
#pragma unroll
            for (int e = 1; e < VEC; ++e) t = (er == e) ? v[e] : t;
            const float b = row_value(t, lrr);
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[e] = (col0 + e >= nx) ? b : v[e];
        }
    };

    // raw input rows: 4 floats (G pass) or 4 codes in two dwords (D pass)
    using Raw = typename std::conditional<FP32_IN, float4, uint2>::type;
    auto load_raw = [&](int zz, Raw &v) STAR_INLINE {
        const size_t off = (size_t)clampi(min(zz, zlast), nz) * plane + (size_t)yc * nx + cl;
        if constexpr (FP32_IN)
            v = *reinterpret_cast<const float4 *>(a.a_in + off);
        else
            v = *reinterpret_cast<const uint2 *>(a.d_in + off);
    };
    auto load_g = [&](int zz, uint2 &v) STAR_INLINE {
        const size_t off = (size_t)clampi(zz, nz) * plane + (size_t)yc * nx + cl;
        v = *reinterpret_cast<const uint2 *>(a.g + off);
    };
    // Exponents of the storage tiles this block touches, staged in LDS once
    // (no global load inside the plane loop, so the memory counters only
    // ever wait for the data rings).  Tables: 0 = input D, 1 = G, 2 = output.
    const int ptx0 = max(xs, 0) >> kTileShift, ptx1 = min(xs + W - 1, nx - 1) >> kTileShift;
    const int pty0 = clampi(ty0 - R, ny) >> kTileShift;
    const int pty1 = clampi(ty0 - R + nt - 1, ny) >> kTileShift;
    const int ptz0 = clampi(zstart, nz) >> kTileShift, ptz1 = clampi(zlast + NR, nz) >> kTileShift;
    const int enx = ptx1 - ptx0 + 1, eny = pty1 - pty0 + 1, enz = ptz1 - ptz0 + 1;
    const int ecount = enx * eny * enz;  // <= 5 * 2 * (lz/64 + 3)
    int *etab = reinterpret_cast<int *>(lds + (size_t)2 * nt * W);
    if constexpr (!FP32_IN) {
        for (int i = threadIdx.x; i < 3 * ecount; i += blockDim.x) {
            const int tbl = i / ecount, k = i % ecount;
            const int gx = ptx0 + k % enx, gy = pty0 + (k / enx) % eny, gz = ptz0 + k / (enx * eny);
            const int *src_tab = tbl == 0 ? a.e_in : tbl == 1 ? a.e_g : a.e_out;
            etab[i] = src_tab[(gz * a.tny + gy) * a.tnx + gx];
        }
        __syncthreads();
    }
    const int exy = ((yc >> kTileShift) - pty0) * enx + ((cl >> kTileShift) - ptx0);
    auto exponent = [&](int tbl, int zz) STAR_INLINE -> int {
        const int tz = (clampi(zz, nz) >> kTileShift) - ptz0;
        return etab[tbl * ecount + tz * enx * eny + exy];
    };
    auto decode4 = [&](const uint2 &q, int e, float (&v)[VEC]) STAR_INLINE {
        v[0] = decode_code<MODE>(q.x & 0xFFFFu, e);
        v[1] = decode_code<MODE>(q.x >> 16, e);
        v[2] = decode_code<MODE>(q.y & 0xFFFFu, e);
        v[3] = decode_code<MODE>(q.y >> 16, e);
    };

    Raw raw[NR];
    int eraw[NR];  // exponent of each raw slot's plane, read from LDS with its load
    uint2 graw[NR];
    float win[P][VEC];
#pragma unroll
    for (int p = 0; p < P; ++p)
#pragma unroll
        for (int e = 0; e < VEC; ++e) win[p][e] = 0.0f;
    // z-segments are whole 64-plane storage tiles (the launcher checks lz),
    // so a lane's running maximum is published at each tile's last plane.
    float runmax = 0.0f, runmax_all = 0.0f;

    // The input ring runs NR planes ahead: a slot is refilled right after
    // its plane entered the window.  The G ring is consumed at the end of a
    // step, so it runs NR-1 planes ahead and its last slot is filled by the
    // first iteration.
    static_for<0, NR>([&](auto phc) STAR_INLINE {
        constexpr int PH = decltype(phc)::value;
        load_raw(zstart + PH, raw[PH]);
        if constexpr (!FP32_IN) eraw[PH] = exponent(0, min(zstart + PH, zlast));
        if constexpr (HAS_G) {
            if constexpr (PH < NR - 1) {
                if (!load_only) load_g(zstart - R + PH, graw[PH]);
            }
        }
    });

    // Publish the running maxima of the output tile holding plane rz: one
    // atomic per wavefront and tile (the lanes of a tile reduce first;
    // non-negative floats order as integers).  Wave-uniform control flow.
    auto publish = [&](int rz) STAR_INLINE {
        const bool has = row_out && col0 >= out_lo && col0 + VEC <= out_hi;
        const int tile = has ? tile_xy + (rz >> kTileShift) * tile_zstride : -1;
        const unsigned v = __float_as_uint(runmax_all);
        bool done = !has;
        for (;;) {  // one trip per distinct tile among the lanes (at most 64)
            const uint64_t act = __ballot(!done);
            if (act == 0) break;
            const int leader = __builtin_ctzll(act);
            const int t0 = __builtin_amdgcn_readlane(tile, leader);
            const bool grp = !done && tile == t0;
            unsigned m = grp ? v : 0u;
#pragma unroll
            for (int sh = 32; sh >= 1; sh >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, sh));
            if (lane == leader) atomicMax(a.max_out + t0, m);
            done = done || grp;
        }
        runmax_all = 0.0f;
    };

    auto step_plane = [&](auto phc, int n) STAR_INLINE {
        constexpr int PH = decltype(phc)::value % P;   // window slot
        constexpr int QH = decltype(phc)::value % NR;  // raw ring slot
        const int zl = zstart + n;  // plane entering the window
        const int r = zl - R;       // plane produced
        const int b = n & 1;
        // The entering plane (loaded NR iterations ago) takes the window slot
        // of the plane that left it; its raw slot is refilled at once.
        if constexpr (FP32_IN) {
            win[PH][0] = raw[QH].x; win[PH][1] = raw[QH].y;
            win[PH][2] = raw[QH].z; win[PH][3] = raw[QH].w;
        } else {
            decode4(raw[QH], eraw[QH], win[PH]);
        }
        xfix(win[PH]);
        load_raw(zl + NR, raw[QH]);
        if constexpr (!FP32_IN) eraw[QH] = exponent(0, min(zl + NR, zlast));
        // G of the plane produced NR-1 steps from now, into the slot the
        // previous step consumed
        constexpr int QN = (QH + NR - 1) % NR;
        if constexpr (HAS_G) {
            if (!load_only) load_g(r + NR - 1, graw[QN]);  // only computing rows use G
        }
        // the centre plane (entered the window R iterations ago) to LDS
        lds_write_row4(lds_row(b, trow), lr, win[(PH - R + P) % P]);
        __syncthreads();
        if (load_only) return;
        // the first plane an output needs (z0) is produced 2R planes into
        // the stream; earlier planes are wind-up that nothing reads
        if (n < 2 * R) return;
        constexpr int CS = (PH - R + P) % P;
        float left[R + 1], right[R + 1];
#pragma unroll
        for (int k = 1; k <= R; ++k) {
            left[k] = from_lower_lane(win[CS][VEC - k], win[CS][0]);
            right[k] = from_upper_lane(win[CS][k - 1], win[CS][VEC - 1]);
        }
        float acc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = a.cf.c[0] * win[CS][e];
#pragma unroll
        for (int i = 1; i <= R; ++i) {
            if (i > 1) __builtin_amdgcn_sched_barrier(0);
            float sv[VEC], nv[VEC];
            lds_read_row4(lds_row(b, tile_row(y - i)), lr, sv);
            lds_read_row4(lds_row(b, tile_row(y + i)), lr, nv);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const float wv = (e - i >= 0) ? win[CS][e - i] : left[i - e];
                const float ev = (e + i < VEC) ? win[CS][e + i] : right[e + i - VEC + 1];
                acc[e] = __builtin_fmaf(a.cf.c[coef_index<3>(kW, i)], wv, acc[e]);
                acc[e] = __builtin_fmaf(a.cf.c[coef_index<3>(kE, i)], ev, acc[e]);
                acc[e] = __builtin_fmaf(a.cf.c[coef_index<3>(kS, i)], sv[e], acc[e]);
                acc[e] = __builtin_fmaf(a.cf.c[coef_index<3>(kN, i)], nv[e], acc[e]);
                acc[e] = __builtin_fmaf(a.cf.c[coef_index<3>(kB, i)], win[(CS - i + P) % P][e], acc[e]);
                if (i < R)
                    acc[e] = __builtin_fmaf(a.cf.c[coef_index<3>(kA, i)], win[(CS + i) % P][e], acc[e]);
            }
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e)
            acc[e] = __builtin_fmaf(a.cf.c[coef_index<3>(kA, R)], win[(CS + R) % P][e], acc[e]);
        const bool ok = row_out && r >= z0 && r < z1 && col0 >= out_lo && col0 + VEC <= out_hi;
        if constexpr (FP32_IN) {
            // G = S A - A
            float g[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                g[e] = acc[e] - win[CS][e];
                runmax = fmaxf(runmax, fabsf(g[e]));
            }
            // one descriptor per plane (wave-uniform); the row goes into the offset
            const auto st = buffer_rsrc(a.g_out + (size_t)clampi(r, nz) * plane, (int)(plane * 4));
            buffer_store4(st, masked_offset((yc * nx + col0) * 4, ok), g[0], g[1], g[2], g[3]);
        } else {
            float gv[VEC] = {0.0f, 0.0f, 0.0f, 0.0f};
            if constexpr (HAS_G) decode4(graw[QH], exponent(1, r), gv);
            const int eo = exponent(2, r);
            uint32_t q[VEC];
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const float v = HAS_G ? acc[e] + gv[e] : acc[e];
                q[e] = encode_code<MODE>(v, eo);
                runmax = fmaxf(runmax, fabsf(v));  // the value before rounding
            }
            const auto st = buffer_rsrc(a.d_out + (size_t)clampi(r, nz) * plane, (int)(plane * 2));
            const v2i packed = {(int)(q[0] | (q[1] << 16)), (int)(q[2] | (q[3] << 16))};
            __builtin_amdgcn_raw_buffer_store_b64(packed, st, masked_offset((yc * nx + col0) * 2, ok),
                                                  0, 0);
        }
        if (!ok) runmax = 0.0f;  // only cells this lane writes count
        runmax_all = fmaxf(runmax_all, runmax);
        runmax = 0.0f;
        // a segment may span several storage tiles in z
        if (((r + 1) & ((1 << kTileShift) - 1)) == 0 && r >= z0 && r < z1 - 1) publish(r);
    };

    int n0 = 0;
    for (; n0 + U <= niter; n0 += U) {
        static_for<0, U>([&](auto phc) STAR_INLINE { step_plane(phc, n0 + decltype(phc)::value); });
    }
    static_for<0, U>([&](auto phc) STAR_INLINE {
        if (n0 + decltype(phc)::value < niter) step_plane(phc, n0 + decltype(phc)::value);
    });
    if (!load_only) publish(z1 - 1);
}

template <int WL, int MODE, bool HAS_G, int NR>
hipError_t launch_m(const LowpArgs &a, hipStream_t stream) {
    constexpr int R = STAR_R;
    constexpr int W = WL * VEC;
    const int nt = a.nw * (64 / WL);
    const int ty = nt - 2 * R;
    if (ty < 1 || a.nw > 16 || a.nw < 1 || a.nx % 4 != 0) return hipErrorInvalidValue;
    int hx = 0, tx = a.nx, ntx = 1;
    if (a.nx > W || WL != 64) {
        hx = (R + VEC - 1) / VEC * VEC;
        tx = W - 2 * hx;
        ntx = (a.nx + tx - 1) / tx;
    }
    const int nty = (a.ny + ty - 1) / ty;
    const int nseg = (a.nz + a.lz - 1) / a.lz;
    const int64_t blocks = (int64_t)ntx * nty * nseg;
    // + the staged exponent tables: 3 tables of (W/64+1) x 2 x (lz/64+3) tiles
    const size_t etab = (size_t)3 * (W / 64 + 1) * 2 * (a.lz / 64 + 3) * sizeof(int);
    const size_t lds = (size_t)2 * nt * W * sizeof(float) + etab;
    if (blocks > ((int64_t)1 << 30) || lds > 160 * 1024) return hipErrorInvalidValue;
    if ((int64_t)a.nx * a.ny * (int64_t)sizeof(float) >= ((int64_t)1 << 31)) return hipErrorInvalidValue;
    auto kern = lowp3d_step<R, WL, MODE, HAS_G, NR>;
    hipError_t e = hipFuncSetAttribute((const void *)kern,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(a.nw * 64), lds, stream, a, hx, tx, ntx,
                       nty);
    return hipGetLastError();
}

template <int WL, int NR>
hipError_t launch_mode(const LowpArgs &a, int mode, hipStream_t stream) {
    if (mode == 0) return launch_m<WL, 0, false, NR>(a, stream);
    if (mode == kCodecF16) return launch_m<WL, kCodecF16, true, NR>(a, stream);
    if (mode == kCodecBF16) return launch_m<WL, kCodecBF16, true, NR>(a, stream);
    if (mode == kScaledPass + kCodecF16) return launch_m<WL, kCodecF16, false, NR>(a, stream);
    if (mode == kScaledPass + kCodecBF16) return launch_m<WL, kCodecBF16, false, NR>(a, stream);
    return hipErrorInvalidValue;
}

template <int WL>
hipError_t launch_d(const LowpArgs &a, int mode, hipStream_t stream) {
    return launch_mode<WL, default_ring<STAR_R>()>(a, mode, stream);
}

}  // namespace

#define STAR_CAT2(a, b) a##b
#define STAR_CAT(a, b) STAR_CAT2(a, b)

hipError_t STAR_CAT(launch_lowp3d_r, STAR_R)(const LowpArgs &a, int mode, hipStream_t stream) {
    // z-segments of whole storage tiles (the kernel publishes per-tile maxima)
    if (a.lz < 1 || a.lz % (1 << kTileShift) != 0 || a.nx < 4 || a.ny < 1 || a.nz < 1)
        return hipErrorInvalidValue;
    if (a.wl == 64) return launch_d<64>(a, mode, stream);
    if (a.wl == 32) return launch_d<32>(a, mode, stream);
    return hipErrorInvalidValue;
}

}  // namespace star
