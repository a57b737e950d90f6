// star3d_rows.hpp -- 3D single-step pass with whole rows per wavefront and no LDS.
//
// The xy-tile kernel (star3d_body.hpp) shares each plane's rows between the
// wavefronts of a workgroup through LDS, which costs a barrier per plane and
// leaves one workgroup per CU waiting on it; its tiles also carry halo
// rows and columns that are loaded but not written.  For one time step
// per pass (K = 1) this form drops both:
//   * A wavefront owns RPL consecutive grid rows of a 256-column strip
//     (64 lanes x 4 cells); every column it holds is an output column and
//     all its rows are output rows.  Strips start at multiples of 256.
//   * z is streamed (Sec. III.A, 2.5D blocking): the lane keeps the last
//     2R+1 planes of its own cells in a register ring (the z-neighbours),
//     with D planes in flight ahead.
//   * y-neighbours: rows within the wavefront's own RPL rows come from its
//     registers; the 2R rows above and below are loaded for the centre
//     plane only (they were loaded moments earlier as the own rows of the
//     neighbouring wavefronts, so they come from the caches).
//   * x-neighbours: from the lane's own cells and the adjacent lanes by DPP
//     wave shifts; the lanes at the strip's ends take the cells beyond the
//     strip from a halo of up to 8 cells per side that only those two
//     lanes load (the DPP "old" operand of the lane with no source).
//   * Narrow grids (LPR = 16 lanes per row): the wavefront is split into
//     four 16-lane row groups, each owning one grid row of a 64-column
//     strip (four consecutive rows per wavefront); x-shifts stay inside
//     each 16-lane DPP row, and each group's end lanes load its halo.
//     Grids a few dozen cells wide then keep most lanes busy.
//   * Wavefronts are independent: no LDS, no barrier; latency is hidden by
//     the other wavefronts on the SIMD.
//   * Clamp boundary (Sec. III.B): plane and row indices are clamped when
//     loaded (wave-uniform, scalar); columns beyond nx take column nx-1
//     (RAGGED form, the strip that crosses nx; or per-element clamped loads
//     when rows are not 16-byte aligned); the halo of the first and last
//     strip repeats the border column.
//   * Each cell is c_C*f_C followed by one FMA per neighbour in coefficient
//     order (W, E, S, N, B, A for i = 1..R), the library-wide order, so the
//     result is bitwise that of every other kernel.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace star {
namespace s3r {

constexpr int VEC = 4;
constexpr int STRIP = 64 * VEC;  // columns per wavefront strip (64 lanes per row)

// One wavefront's work: `rows0` .. rows0+RPL-1 of strip `strip`, planes
// z0 .. min(z0+lz, nz)-1.  Every argument is wave-uniform.
// LPR: lanes per row, 64 (one row group, strips of 256 columns) or 16
// (four row groups, strips of 64 columns; group g owns rows
// rows0 + g*RPL ..; one row per group, radius <= 4, no neighbour prefetch).
// NBP: the y-neighbour rows and the halo of the next centre plane are
// loaded one plane ahead (more registers, latency off the critical path).
// SYM: shared coefficients, one per axis and distance (cf holds c_C, then
// c_x,i, c_y,i, c_z,i for i = 1..R): per distance and axis one FMA with the
// rounded sum of the pair of cells.
// pad > 0: padded-halo boundary (Sec. IV.B): the grid is the padded array
// and the cells of its frame of `pad` cells keep their values.
template <int R, int RPL, int D, bool NBP, bool ALIGNED, bool RAGGED, bool SYM = false,
          int LPR = 64>
__device__ __forceinline__ void star3d_rows_body(const float *__restrict__ src,
                                                 float *__restrict__ dst, int nx, int ny, int nz,
                                                 int strip, int rows0, int z0, int lz,
                                                 const Coefs &cf, int pad = 0) {
    constexpr int P = 2 * R + 1;       // z-window planes
    constexpr int NQ = P + D;          // ring: window plus D planes in flight
    constexpr int HW = R > 4 ? 8 : 4;  // halo cells per side
    constexpr int NB = NBP ? 2 : 1;    // neighbour buffers (current, next)
    static_assert(R <= 2 * VEC, "x-neighbours come from the lanes at most two away");
    static_assert(LPR == 64 || (LPR == 16 && RPL == 1 && R <= VEC && !NBP),
                  "16-lane rows: one row per group, radius <= 4, no neighbour prefetch");
    constexpr int SW = LPR * VEC;      // strip width in columns

    const int lane = threadIdx.x & 63;
    const int gl = lane & (LPR - 1);   // lane within its row group
    const int y0 = LPR == 64 ? rows0 : rows0 + (lane / LPR) * RPL;  // the group's first row
    const int x0 = strip * SW;
    const int col0 = x0 + gl * VEC;
    const int z1 = min(z0 + lz, nz);
    const int zstart = z0 - R;          // first plane streamed
    const int niter = (z1 - z0) + 2 * R;
    const int zlast = zstart + niter - 1;
    const size_t plane = (size_t)nx * (size_t)ny;
    const int plane_bytes = (int)(plane * sizeof(float));  // < 2^31, checked by the launcher
    const bool first_strip = x0 == 0;
    const bool last_strip = x0 + SW >= nx;

    // Row `yy` (clamped to the grid) of plane `zz` (clamped), this lane's 4 cells.
    auto load_row = [&](int zz, int yy, float (&v)[VEC]) STAR_INLINE {
        const float *row = src + (size_t)clampi(zz, nz) * plane + (size_t)clampi(yy, ny) * nx;
        if constexpr (ALIGNED) {
            const float4 t = *reinterpret_cast<const float4 *>(row + min(col0, nx - VEC));
            v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[e] = row[clampi(col0 + e, nx)];
        }
    };
    // Columns beyond nx take column nx-1.  With 16-byte rows (nx % 4 == 0)
    // a lane is either inside or wholly beyond; beyond, its clamped load
    // holds columns nx-4 .. nx-1, so column nx-1 is its element 3.
    auto xfix = [&](float (&v)[VEC]) STAR_INLINE {
        if constexpr (ALIGNED && RAGGED) {
            const bool beyond = col0 >= nx;
#pragma unroll
            for (int e = 0; e < VEC - 1; ++e) v[e] = beyond ? v[VEC - 1] : v[e];
        }
    };

    // Halo cells of row yy, plane zz, held by the row group's two end lanes
    // in one register set: its first lane gets columns x0-HW .. x0-1 (the
    // cells left of the strip), its last lane x0+SW .. x0+SW+HW-1 (right of it);
    // other lanes' values are never read.  The first strip's left halo and
    // the last strip's right halo are the border column, which the end lane
    // holds itself (filled in at use).
    auto load_halo = [&](int zz, int yy, float (&h)[HW]) STAR_INLINE {
        const float *row = src + (size_t)clampi(zz, nz) * plane + (size_t)clampi(yy, ny) * nx;
        if ((gl == 0 && !first_strip) || (gl == LPR - 1 && !last_strip)) {
            const int c0 = gl == 0 ? x0 - HW : x0 + SW;
            if constexpr (ALIGNED) {
                // 16-byte columns: x0 - HW >= 0 and x0 + SW <= nx - 4 here
#pragma unroll
                for (int c = 0; c < HW / VEC; ++c) {
                    const float4 t = *reinterpret_cast<const float4 *>(row + min(c0 + VEC * c, nx - VEC));
                    h[VEC * c] = t.x; h[VEC * c + 1] = t.y; h[VEC * c + 2] = t.z; h[VEC * c + 3] = t.w;
                }
                if constexpr (HW > VEC) {
                    // the second vector of the right halo may lie beyond nx
                    if (gl == LPR - 1 && c0 + VEC >= nx) {
#pragma unroll
                        for (int j = VEC; j < HW; ++j) h[j] = h[VEC - 1];
                    }
                }
            } else {
#pragma unroll
                for (int j = 0; j < HW; ++j) h[j] = row[clampi(c0 + j, nx)];
            }
        }
    };

    float q[NQ][RPL][VEC];           // own rows, ring of planes
    float nb[NB][2 * R][VEC];        // rows y0-R .. y0-1, y0+RPL .. y0+RPL+R-1
    float h[NB][RPL][HW];            // halo of each own row (end lanes only)
#pragma unroll
    for (int p = 0; p < NQ; ++p)
#pragma unroll
        for (int k = 0; k < RPL; ++k)
#pragma unroll
            for (int e = 0; e < VEC; ++e) q[p][k][e] = 0.0f;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int k = 0; k < RPL; ++k)
#pragma unroll
            for (int j = 0; j < HW; ++j) h[b][k][j] = 0.0f;

    auto load_plane = [&](int zz, float (&v)[RPL][VEC]) STAR_INLINE {
#pragma unroll
        for (int k = 0; k < RPL; ++k) load_row(min(zz, zlast), y0 + k, v[k]);
    };
    // y-neighbour rows and halo of centre plane zc into buffer B
    auto load_centre = [&](int zc, auto bc) STAR_INLINE {
        constexpr int B = decltype(bc)::value;
#pragma unroll
        for (int j = 0; j < R; ++j) {
            load_row(zc, y0 - R + j, nb[B][j]);
            load_row(zc, y0 + RPL + j, nb[B][R + j]);
        }
#pragma unroll
        for (int k = 0; k < RPL; ++k) load_halo(zc, y0 + k, h[B][k]);
    };

    static_for<0, D>([&](auto phc) STAR_INLINE {
        constexpr int PH = decltype(phc)::value;
        load_plane(zstart + PH, q[PH]);
    });
    if constexpr (NBP) load_centre(z0, std::integral_constant<int, 0>{});

    // Output cells of own row k from centre slot CS (plane r), buffer b.
    auto cells = [&](auto csc, int k, auto bc, float (&res)[VEC]) STAR_INLINE {
        constexpr int CS = decltype(csc)::value;
        constexpr int b = decltype(bc)::value;
        const float(&c)[VEC] = q[CS][k];
        // the end lanes' halo; the first and last strip repeat their own
        // border cell
        float hlk[HW], hrk[HW];
#pragma unroll
        for (int j = 0; j < HW; ++j) {
            hlk[j] = first_strip ? c[0] : h[b][k][j];
            hrk[j] = last_strip ? c[VEC - 1] : h[b][k][j];
        }
        // left[m]: column col0 - m; right[m]: column col0 + VEC - 1 + m
        float left[R + 1], right[R + 1];
#pragma unroll
        for (int m = 1; m <= R; ++m) {
            if (m <= VEC) {
                left[m] = from_lower_lane_in<LPR>(c[VEC - m], hlk[HW - m]);
                right[m] = from_upper_lane_in<LPR>(c[m - 1], hrk[m - 1]);
            } else {  // two lanes away: lane 1 takes lane 0's halo via the first shift
                left[m] = from_lower_lane(from_lower_lane(c[2 * VEC - m], hlk[HW + VEC - m]),
                                          hlk[HW - m]);
                right[m] = from_upper_lane(from_upper_lane(c[m - VEC - 1], hrk[m - VEC - 1]),
                                           hrk[m - 1]);
            }
        }
        // row k +- i: own row, or one of the loaded neighbour rows
        auto yrow = [&](int d) STAR_INLINE -> const float(&)[VEC] {
            const int kk = k + d;
            if (kk < 0) return nb[b][R + kk];
            if (kk >= RPL) return nb[b][R + (kk - RPL)];
            return q[CS][kk];
        };
        float acc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = cf.c[0] * c[e];
#pragma unroll
        for (int i = 1; i <= R; ++i) {
            const float(&sv)[VEC] = yrow(-i);
            const float(&nv)[VEC] = yrow(i);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const float wv = (e - i >= 0) ? c[e - i] : left[i - e];
                const float ev = (e + i < VEC) ? c[e + i] : right[e + i - VEC + 1];
                const float bv = q[(CS - i + NQ) % NQ][k][e], av = q[(CS + i) % NQ][k][e];
                if constexpr (SYM) {
                    acc[e] = __builtin_fmaf(cf.c[1 + 3 * (i - 1)], wv + ev, acc[e]);
                    acc[e] = __builtin_fmaf(cf.c[2 + 3 * (i - 1)], sv[e] + nv[e], acc[e]);
                    acc[e] = __builtin_fmaf(cf.c[3 + 3 * (i - 1)], bv + av, acc[e]);
                } else {
                    acc[e] = __builtin_fmaf(cf.c[coef_index<3>(kW, i)], wv, acc[e]);
                    acc[e] = __builtin_fmaf(cf.c[coef_index<3>(kE, i)], ev, acc[e]);
                    acc[e] = __builtin_fmaf(cf.c[coef_index<3>(kS, i)], sv[e], acc[e]);
                    acc[e] = __builtin_fmaf(cf.c[coef_index<3>(kN, i)], nv[e], acc[e]);
                    acc[e] = __builtin_fmaf(cf.c[coef_index<3>(kB, i)], bv, acc[e]);
                    acc[e] = __builtin_fmaf(cf.c[coef_index<3>(kA, i)], av, acc[e]);
                }
            }
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) res[e] = acc[e];
    };

    // Padded-halo frame: a frame cell (element e of own row k, plane r)
    // keeps its centre value ctr; other cells keep v.
    auto frame_value = [&](int r, int k, int e, float ctr, float v) STAR_INLINE -> float {
        const int yy = y0 + k, cc = col0 + e;
        return (r < pad || r >= nz - pad || yy < pad || yy >= ny - pad || cc < pad ||
                cc >= nx - pad) ? ctr : v;
    };

    auto store_row = [&](int r, int k, const float (&res)[VEC]) STAR_INLINE {
        const int yy = y0 + k;
        const bool ok_row = yy < ny && r >= z0 && r < z1;
        const auto rs = buffer_rsrc(dst + (size_t)clampi(r, nz) * plane, plane_bytes);
        const int rowoff = clampi(yy, ny) * nx;
        if constexpr (ALIGNED) {
            const bool ok = ok_row && col0 < nx;
            // non-temporal: keeps L2 for the neighbour rows (measured on
            // 512^3: +4..7 % at R = 1, 3, 6, 8)
            buffer_store4<kStoreNT>(rs, ok ? (rowoff + col0) * 4 : kOutOfRange, res[0], res[1],
                                    res[2], res[3]);
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const bool ok = ok_row && col0 + e < nx;
                buffer_store1<kStoreNT>(rs, ok ? (rowoff + col0 + e) * 4 : kOutOfRange, res[e]);
            }
        }
    };

    // Iteration n: plane zl = zstart + n enters the window (ring slot n % NQ,
    // loaded D iterations ago); plane zl + D is requested; the centre plane
    // r = zl - R is computed once its window is complete (n >= 2R).  With
    // NBP the neighbour buffer alternates with n, so the unrolled trip is
    // even and the buffer index compile-time (n0 is a multiple of U).
    constexpr int U = (NBP && NQ % 2 == 1) ? 2 * NQ : NQ;
    auto step_plane = [&](auto phc, int n) STAR_INLINE {
        constexpr int PH = decltype(phc)::value % NQ;
        constexpr int B = NBP ? (decltype(phc)::value & 1) : 0;
        const int zl = zstart + n;
        load_plane(zl + D, q[(PH + D) % NQ]);
#pragma unroll
        for (int k = 0; k < RPL; ++k) xfix(q[PH][k]);
        if (n < 2 * R) return;
        const int r = zl - R;
        constexpr int CS = (PH - R + NQ) % NQ;
        if constexpr (NBP) {
            // the first centre plane (n = 2R, even) was loaded into buffer 0
            if (r + 1 < z1) load_centre(r + 1, std::integral_constant<int, B ^ 1>{});
        } else {
            load_centre(r, std::integral_constant<int, 0>{});
        }
#pragma unroll
        for (int k = 0; k < RPL; ++k) {
            float res[VEC];
            cells(std::integral_constant<int, CS>{}, k, std::integral_constant<int, B>{}, res);
            if (pad > 0) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) res[e] = frame_value(r, k, e, q[CS][k][e], res[e]);
            }
            store_row(r, k, res);
        }
    };

    int n0 = 0;
    for (; n0 + U <= niter; n0 += U) {
        static_for<0, U>([&](auto phc) STAR_INLINE { step_plane(phc, n0 + decltype(phc)::value); });
    }
    static_for<0, U>([&](auto phc) STAR_INLINE {
        if (n0 + decltype(phc)::value < niter) step_plane(phc, n0 + decltype(phc)::value);
    });
}

// Planes in flight per wavefront: enough to cover the memory latency at
// R <= 2; from R = 3 on one plane, which shortens the time between a
// wavefront loading its own row and its neighbours reading that row back
// from L2 (512^3, R = 3, two rows per wavefront: 530 -> 547 GCell/s; equal
// elsewhere).  Two planes from R = 3 on: four rows per wavefront at R = 3, 4
// 555 -> 546 and 525 -> 513 (and 12 bytes of scratch per lane at R = 4),
// two rows at R = 5, 6 402 -> 399 and 365 -> 359 GCell/s.
template <int R, int RPL>
constexpr int prefetch_rows3() {
    return R <= 2 ? (RPL == 1 ? 6 : 3) : 1;
}

}  // namespace s3r
}  // namespace star
