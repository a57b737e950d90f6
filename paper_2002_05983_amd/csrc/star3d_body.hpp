// star3d_body.hpp -- 3D star stencil: xy tile in LDS, z streamed, K fused steps.
//
// The per-workgroup body shared by the single-grid kernel and the batched
// work-list kernel.
//
// Method (Sec. III.A of the paper: 2.5D spatial blocking -- block x and y,
// stream z -- combined with temporal blocking by a chain of K stages and
// overlapped halos, Eq. (2)):
//   * A workgroup owns an xy tile: NW wavefronts of 64/WL tile rows each.
//     WL lanes of a wavefront hold VEC consecutive cells each, so a row spans
//     WL*VEC columns.  With WL = 64, a grid at most that wide is one tile and
//     needs no x halo; otherwise tiles overlap by Hx = roundup(K*R, VEC)
//     columns per side (the lanes at the ends of a row then hold halo cells,
//     so a DPP shift that crosses from one row into the next only ever
//     feeds halo cells).
//   * Rows: the tile's TY output rows, (K-1)*R computed halo rows per side
//     (stages 1..K-1 produce the values the next stage's halo needs), and R
//     load-only rows per side that only supply stage 1's y-neighbours.
//   * z is streamed.  Stage s (1..K) runs R planes behind stage s-1 and
//     starts 2*s*R planes into the stream, at its first needed plane; each
//     stage keeps the last 2R+1 planes of its input column in registers (the
//     z-neighbours).  Per plane, every stage writes its centre plane row to
//     LDS (double-buffered), one barrier, then reads its y-neighbours from
//     LDS, its x-neighbours from its own and adjacent lanes (DPP wave
//     shifts), and applies one step.  Only stage K is written back.
//   * Clamp boundary (Sec. III.B) at every stage: y-neighbour rows are
//     clamped to the grid when read from LDS; z planes before the grid are
//     filled with a stage's plane 0 when it is produced, planes after it
//     repeat plane nz-1; columns outside [0, nx) take the border column.
//   * Each cell is c_C*f_C followed by one FMA per neighbour in coefficient
//     order (W, E, S, N, B, A for i = 1..R), the library-wide order.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace star {
namespace s3d {

// LDS row layout: chunk-major, [VEC/4][WL lanes][4 floats], so that every
// 128-bit LDS access of a row's lanes covers consecutive addresses.
template <int VEC, int WL>
__device__ __forceinline__ int lds_off(int lr, int chunk) {
    return (chunk * WL + lr) * 4;
}

template <int VEC, int WL>
__device__ __forceinline__ void lds_write_row(float *row, int lr, const float (&v)[VEC]) {
#pragma unroll
    for (int c = 0; c < VEC / 4; ++c)
        *reinterpret_cast<float4 *>(row + lds_off<VEC, WL>(lr, c)) =
            make_float4(v[4 * c], v[4 * c + 1], v[4 * c + 2], v[4 * c + 3]);
}

template <int VEC, int WL>
__device__ __forceinline__ void lds_read_row(const float *row, int lr, float (&v)[VEC]) {
#pragma unroll
    for (int c = 0; c < VEC / 4; ++c) {
        const float4 t = *reinterpret_cast<const float4 *>(row + lds_off<VEC, WL>(lr, c));
        v[4 * c] = t.x; v[4 * c + 1] = t.y; v[4 * c + 2] = t.z; v[4 * c + 3] = t.w;
    }
}

// One workgroup's work: x-strip `strip`, tile row band `ytile` and
// z-segment `zseg` of one grid (all block-uniform).  Uses the dynamic LDS
// and one barrier per plane.  EDGE = false is the interior form for a tile
// whose columns, rows and planes stay inside the grid at every stage
// (star3d_interior): no clamp is ever applied and the border code is left
// out; for such a tile it computes the same bits as the general form.
// PAIR (single-step passes only): two planes per barrier -- both centre
// rows go to LDS (four buffers), then both planes are computed -- which
// halves the barriers and the per-plane synchronisation; the same bits.
// pad > 0: padded-halo boundary (Sec. IV.B): the grid is the padded array
// and its frame of `pad` cells is fixed; in the general form every stage
// gives a frame cell its own (unchanged) value, and the interior test
// (star3d_interior) keeps frame cells out of the interior form.
template <int R, int K, int VEC, int WL, int D, bool ALIGNED, bool EDGE = true, bool PAIR = false>
__device__ __forceinline__ void star3d_body(const float *__restrict__ src, float *__restrict__ dst,
                                            int nx, int ny, int nz, int hx, int tx, int strip,
                                            int ytile, int zseg, int lz, const Coefs &cf,
                                            int pad = 0) {
    static_assert(!PAIR || K == 1, "two planes per barrier: single-step passes only");
    constexpr int P = 2 * R + 1;      // planes a stage keeps: its z-window
    // Single-step passes load straight into an input ring of the window plus
    // D planes in flight (plus one in the paired form, whose second load
    // would otherwise overwrite the first plane's oldest window plane).
    // Passes of K > 1 steps keep the input ring at the window (P planes) and
    // land their loads in a separate staging ring of D planes, moved into
    // the window when consumed: every ring then turns with a period dividing
    // lcm(P, D), which keeps the unrolled loop one or two windows long
    // whatever D is.
    constexpr bool STAGED = K > 1;
    constexpr int NQ = STAGED ? P : P + D + (PAIR ? 1 : 0);
    constexpr int DIST = D;           // prefetch distance in planes
    // Unrolled planes per loop trip: every ring index must be compile-time,
    // so the trip covers a whole number of turns of each ring (and, paired,
    // a whole number of pairs).
    constexpr int U = PAIR ? (NQ % 2 == 0 ? NQ : 2 * NQ) : (K == 1) ? NQ : P * D / gcd_i(P, D);
    constexpr int RPW = 64 / WL;      // tile rows per wavefront
    constexpr int W = WL * VEC;       // columns per tile row
    constexpr int ROWF = W;           // floats per LDS row
    static_assert(R <= 2 * VEC && VEC % 4 == 0 && 64 % WL == 0, "bad vector width");
    extern __shared__ float lds[];    // [K][2][NT][ROWF]

    const int lane = threadIdx.x & 63;
    const int lr = lane % WL;         // lane within its tile row
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nt = (blockDim.x >> 6) * RPW;  // tile rows
    const int ty = nt - 2 * K * R;    // output rows of the tile
    const int ty0 = ytile * ty;
    const int trow = w * RPW + lane / WL;  // this lane's tile row
    const int y = ty0 - K * R + trow;      // and grid row
    const int yc = clampi(y, ny);
    // Stage s (1-based) is needed on tile rows s*R .. nt-1-s*R (the rows of
    // stage s+1's y-window, or the output rows for s = K); a wavefront
    // computes a stage only when one of its rows is among them.  Rows
    // 0..R-1 and nt-R..nt-1 only feed stage 1: a wavefront made of such
    // rows only loads.
    auto computes = [&](int s) STAR_INLINE {
        return w * RPW + RPW - 1 >= s * R && w * RPW < nt - s * R;
    };
    const bool load_only = !computes(1);
    const int xs = strip * tx - hx;   // first column held by lane 0 of a row
    const int col0 = xs + lr * VEC;
    const int z0 = zseg * lz;
    const int z1 = min(z0 + lz, nz);
    const int zstart = z0 - K * R;
    const int niter = (z1 - z0) + 2 * K * R;
    const int zlast = zstart + niter - 1;
    const bool left_edge = xs < 0;
    const bool right_edge = xs + W > nx;
    const int out_lo = max(xs + hx, 0);
    const int out_hi = min(xs + hx + tx, nx);
    const bool row_out = y >= ty0 && y < ty0 + ty && y < ny;
    const size_t plane = (size_t)nx * (size_t)ny;
    const int plane_bytes = (int)(plane * sizeof(float));  // < 2^31, checked by the launcher

    // LDS row of stage s (0-based), buffer b, tile row r.
    auto lds_row = [&](int s, int b, int r) STAR_INLINE -> float * {
        return lds + ((size_t)((s * 2 + b) * nt + r)) * ROWF;
    };
    // Tile row holding grid row clamp(yy) (clamped into the tile as well).
    auto tile_row = [&](int yy) STAR_INLINE -> int {
        const int r = (EDGE ? clampi(yy, ny) : yy) - (ty0 - K * R);
        return r < 0 ? 0 : (r >= nt ? nt - 1 : r);
    };
    // Value of v in lane `l` of this lane's tile row.
    auto row_value = [&](float v, int l) STAR_INLINE -> float {
        float b = lane_value(v, l);
#pragma unroll
        for (int k = 1; k < RPW; ++k) b = (lane / WL == k) ? lane_value(v, k * WL + l) : b;
        return b;
    };

    auto xfix = [&](float (&v)[VEC]) STAR_INLINE {
        if constexpr (!EDGE) return;
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

    auto load_plane = [&](int zz, float (&v)[VEC]) STAR_INLINE {
        const float *row =
            src + (size_t)(EDGE ? clampi(min(zz, zlast), nz) : min(zz, zlast)) * plane + (size_t)yc * nx;
        if constexpr (ALIGNED) {
#pragma unroll
            for (int c = 0; c < VEC / 4; ++c) {
                const int cc = EDGE ? min(max(col0 + 4 * c, 0), nx - 4) : col0 + 4 * c;
                const float4 t = *reinterpret_cast<const float4 *>(row + cc);
                v[4 * c] = t.x; v[4 * c + 1] = t.y; v[4 * c + 2] = t.z; v[4 * c + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[e] = row[EDGE ? clampi(col0 + e, nx) : col0 + e];
        }
    };

    // Cells of one stage: centre row ctr, queue q (z-window, NS slots, centre
    // slot CS), LDS buffer of the centre plane for y-neighbours.
    auto cells = [&](auto nsc, auto csc, const float (&q)[decltype(nsc)::value][VEC], int s,
                     int b, float (&res)[VEC]) STAR_INLINE {
        constexpr int NS = decltype(nsc)::value;
        constexpr int CS = decltype(csc)::value;
        // the wavefront's end lanes take their own border cell (general
        // form) or zero (interior form: they hold halo columns)
        auto lower = [&](float v) STAR_INLINE {
            return EDGE ? from_lower_lane(v, q[CS][0]) : from_lower_lane_or_zero(v);
        };
        auto upper = [&](float v) STAR_INLINE {
            return EDGE ? from_upper_lane(v, q[CS][VEC - 1]) : from_upper_lane_or_zero(v);
        };
        // left[k]: column base - k; right[k]: column base + VEC - 1 + k
        float left[R + 1], right[R + 1];
#pragma unroll
        for (int k = 1; k <= R; ++k) {
            if (k <= VEC) {  // the adjacent lane
                left[k] = lower(q[CS][VEC - k]);
                right[k] = upper(q[CS][k - 1]);
            } else {  // two lanes away (R > VEC)
                left[k] = lower(lower(q[CS][2 * VEC - k]));
                right[k] = upper(upper(q[CS][k - VEC - 1]));
            }
        }
        float acc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = cf.c[0] * q[CS][e];
#pragma unroll
        for (int i = 1; i <= R; ++i) {
            // keep the scheduler from hoisting every distance's LDS reads at
            // once (register pressure at large R)
            if (i > 1) __builtin_amdgcn_sched_barrier(0);
            float sv[VEC], nv[VEC];
            lds_read_row<VEC, WL>(lds_row(s, b, tile_row(y - i)), lr, sv);
            lds_read_row<VEC, WL>(lds_row(s, b, tile_row(y + i)), lr, nv);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const float wv = (e - i >= 0) ? q[CS][e - i] : left[i - e];
                const float ev = (e + i < VEC) ? q[CS][e + i] : right[e + i - VEC + 1];
                acc[e] = __builtin_fmaf(cf.c[coef_index<3>(kW, i)], wv, acc[e]);
                acc[e] = __builtin_fmaf(cf.c[coef_index<3>(kE, i)], ev, acc[e]);
                acc[e] = __builtin_fmaf(cf.c[coef_index<3>(kS, i)], sv[e], acc[e]);
                acc[e] = __builtin_fmaf(cf.c[coef_index<3>(kN, i)], nv[e], acc[e]);
                acc[e] = __builtin_fmaf(cf.c[coef_index<3>(kB, i)], q[(CS - i + NS) % NS][e], acc[e]);
                acc[e] = __builtin_fmaf(cf.c[coef_index<3>(kA, i)], q[(CS + i) % NS][e], acc[e]);
            }
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) res[e] = acc[e];
    };

    float q0[NQ][VEC];
    float stg[STAGED ? D : 1][VEC];
    float q[K > 1 ? K - 1 : 1][P][VEC];
#pragma unroll
    for (int s = 0; s < (K > 1 ? K - 1 : 1); ++s)
#pragma unroll
        for (int p = 0; p < P; ++p)
#pragma unroll
            for (int e = 0; e < VEC; ++e) q[s][p][e] = 0.0f;
#pragma unroll
    for (int p = 0; p < NQ; ++p)
#pragma unroll
        for (int e = 0; e < VEC; ++e) q0[p][e] = 0.0f;

    static_for<0, DIST>([&](auto phc) STAR_INLINE {
        if constexpr (STAGED)
            load_plane(zstart + decltype(phc)::value, stg[decltype(phc)::value]);
        else
            load_plane(zstart + decltype(phc)::value, q0[decltype(phc)::value]);
    });

    // Padded-halo frame: a frame cell (element e of this lane's row, plane
    // r) keeps its centre value ctr; other cells keep v.
    const bool frame_row = y < pad || y >= ny - pad;
    auto frame_value = [&](int r, int e, float ctr, float v) STAR_INLINE -> float {
        const int c = col0 + e;
        return (frame_row || r < pad || r >= nz - pad || c < pad || c >= nx - pad) ? ctr : v;
    };

    // The output row of plane r (stage K), masked to the tile and grid.
    auto store_row = [&](int r, const float (&res)[VEC]) STAR_INLINE {
        // one descriptor per plane (wave-uniform); the row goes into the
        // per-lane offset
        const bool ok_row = row_out && r >= z0 && r < z1;
        const auto rs = buffer_rsrc(dst + (size_t)clampi(r, nz) * plane, plane_bytes);
        const int rowoff = yc * nx;
        if constexpr (ALIGNED) {
#pragma unroll
            for (int c = 0; c < VEC / 4; ++c) {
                const int cc = col0 + 4 * c;
                const bool ok = ok_row && cc >= out_lo && cc + 4 <= out_hi;
                buffer_store4<kStoreNT>(rs, ok ? (rowoff + cc) * 4 : kOutOfRange, res[4 * c], res[4 * c + 1],
                              res[4 * c + 2], res[4 * c + 3]);
            }
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                const int cc = col0 + e;
                const bool ok = ok_row && cc >= out_lo && cc < out_hi;
                buffer_store1<kStoreNT>(rs, ok ? (rowoff + cc) * 4 : kOutOfRange, res[e]);
            }
        }
    };

    auto step_plane = [&](auto phc, int n) STAR_INLINE {
        constexpr int PH = decltype(phc)::value % NQ;  // slot in the input ring
        constexpr int PS = decltype(phc)::value % P;   // slot in the stage windows
        const int zl = zstart + n;  // plane entering stage 1
        const int b = n & 1;        // LDS buffer of this iteration
        if constexpr (STAGED) {
            // plane zl arrived in staging slot n % D; move it into the window
            // and reuse the slot for plane zl + D
            constexpr int PD = decltype(phc)::value % D;
#pragma unroll
            for (int e = 0; e < VEC; ++e) q0[PH][e] = stg[PD][e];
            load_plane(zl + DIST, stg[PD]);
        } else {
            load_plane(zl + DIST, q0[(PH + DIST) % NQ]);
        }
        if constexpr (ALIGNED) xfix(q0[PH]);
        // centre planes of every stage into LDS
        lds_write_row<VEC, WL>(lds_row(0, b, trow), lr, q0[(PH - R + NQ) % NQ]);
        static_for<2, K + 1>([&](auto sc) STAR_INLINE {
            constexpr int S = decltype(sc)::value;
            if (n < 2 * S * R || !computes(S - 1)) return;  // stage S not started (below)
            lds_write_row<VEC, WL>(lds_row(S - 1, b, trow), lr, q[S - 2][(PS - R + P) % P]);
        });
        __syncthreads();
        if (!load_only) {
            static_for<1, K + 1>([&](auto sc) STAR_INLINE {
                constexpr int S = decltype(sc)::value;
                // Stage S first produces a plane that an output depends on at
                // iteration 2*S*R (workgroup-uniform); before that nothing
                // reads what it would produce.  A wavefront none of whose rows
                // stage S needs skips it.
                if (n < 2 * S * R || !computes(S)) return;
                const int r = zl - S * R;  // plane produced by stage S
                float res[VEC];
                if constexpr (S == 1)
                    cells(std::integral_constant<int, NQ>{},
                          std::integral_constant<int, (PH - R + NQ) % NQ>{}, q0, 0, b, res);
                else
                    cells(std::integral_constant<int, P>{},
                          std::integral_constant<int, (PS - R + P) % P>{}, q[S - 2], S - 1, b,
                          res);
                if constexpr (EDGE) {
                    if (pad > 0) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) {
                            float ctr;
                            if constexpr (S == 1)
                                ctr = q0[(PH - R + NQ) % NQ][e];
                            else
                                ctr = q[S - 2][(PS - R + P) % P][e];
                            res[e] = frame_value(r, e, ctr, res[e]);
                        }
                    }
                }
                if constexpr (S < K) {
                    constexpr int WS = PS;
                    if constexpr (EDGE) {
                        if (r >= nz) {
#pragma unroll
                            for (int e = 0; e < VEC; ++e) res[e] = q[S - 1][(WS + P - 1) % P][e];
                        } else {
                            xfix(res);
                        }
                    }
#pragma unroll
                    for (int e = 0; e < VEC; ++e) q[S - 1][WS][e] = res[e];
                    if constexpr (EDGE) {
                        if (r == 0) {
                            static_for<1, R + 1>([&](auto mc) STAR_INLINE {
                                constexpr int MM = decltype(mc)::value;
#pragma unroll
                                for (int e = 0; e < VEC; ++e) q[S - 1][(WS - MM + P) % P][e] = res[e];
                            });
                        }
                    }
                } else {
                    store_row(r, res);
                }
            });
        }
    };

    // Paired form: iterations n (even) and n+1 share one barrier; their
    // centre rows go to LDS buffers b and b+1 (b alternates 0, 2), whose
    // previous readers finished before the last pair's barrier.
    auto step_pair = [&](auto phc, int n) STAR_INLINE {
        constexpr int PH0 = decltype(phc)::value % NQ;
        constexpr int PH1 = (decltype(phc)::value + 1) % NQ;
        const int zl = zstart + n;
        const int b = n & 2;
        load_plane(zl + DIST, q0[(PH0 + DIST) % NQ]);
        load_plane(zl + 1 + DIST, q0[(PH1 + DIST) % NQ]);
        if constexpr (ALIGNED) {
            xfix(q0[PH0]);
            xfix(q0[PH1]);
        }
        lds_write_row<VEC, WL>(lds_row(0, b, trow), lr, q0[(PH0 - R + NQ) % NQ]);
        lds_write_row<VEC, WL>(lds_row(0, b + 1, trow), lr, q0[(PH1 - R + NQ) % NQ]);
        __syncthreads();
        if (load_only) return;
        if (n >= 2 * R) {  // the first plane an output needs comes 2R planes in
            float res[VEC];
            cells(std::integral_constant<int, NQ>{}, std::integral_constant<int, (PH0 - R + NQ) % NQ>{},
                  q0, 0, b, res);
            if constexpr (EDGE) {
                if (pad > 0) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        res[e] = frame_value(zl - R, e, q0[(PH0 - R + NQ) % NQ][e], res[e]);
                }
            }
            store_row(zl - R, res);
        }
        // one plane at a time: interleaving the two would raise the
        // register pressure past the 128-VGPR budget
        __builtin_amdgcn_sched_barrier(0);
        if (n + 1 >= 2 * R && n + 1 < niter) {
            float res[VEC];
            cells(std::integral_constant<int, NQ>{}, std::integral_constant<int, (PH1 - R + NQ) % NQ>{},
                  q0, 0, b + 1, res);
            if constexpr (EDGE) {
                if (pad > 0) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e)
                        res[e] = frame_value(zl + 1 - R, e, q0[(PH1 - R + NQ) % NQ][e], res[e]);
                }
            }
            store_row(zl + 1 - R, res);
        }
    };

    int n0 = 0;
    if constexpr (PAIR) {
        for (; n0 + U <= niter; n0 += U) {
            static_for<0, U / 2>([&](auto pc) STAR_INLINE {
                step_pair(std::integral_constant<int, 2 * decltype(pc)::value>{}, n0 + 2 * decltype(pc)::value);
            });
        }
        static_for<0, U / 2>([&](auto pc) STAR_INLINE {
            if (n0 + 2 * decltype(pc)::value < niter)
                step_pair(std::integral_constant<int, 2 * decltype(pc)::value>{}, n0 + 2 * decltype(pc)::value);
        });
    } else {
        for (; n0 + U <= niter; n0 += U) {
            static_for<0, U>([&](auto phc) STAR_INLINE { step_plane(phc, n0 + decltype(phc)::value); });
        }
        static_for<0, U>([&](auto phc) STAR_INLINE {
            if (n0 + decltype(phc)::value < niter) step_plane(phc, n0 + decltype(phc)::value);
        });
    }
}

// True when a tile needs no clamp at any stage: its columns xs .. xs+W-1,
// its rows ty0-KR .. ty0-KR+nt-1 and the planes z0-2KR .. z1-1+KR its
// stages read and produce all lie inside the grid.
template <int R, int K, int VEC, int WL>
__device__ __forceinline__ bool star3d_interior(int nx, int ny, int nz, int hx, int tx, int strip,
                                                int ytile, int zseg, int lz, int nt, int pad = 0) {
    const int xs = strip * tx - hx;
    const int ty = nt - 2 * K * R;
    const int y0 = ytile * ty - K * R;
    const int z0 = zseg * lz;
    const int z1 = min(z0 + lz, nz);
    return hx > 0 && xs >= pad && xs + WL * VEC <= nx - pad && y0 >= pad && y0 + nt <= ny - pad &&
           z0 > 2 * K * R + pad && z1 + K * R <= nz - pad;
}

// Prefetch depth (planes) per configuration, sized so that a 1024-thread
// workgroup stays within 128 VGPRs per lane: deep for K = 1 (memory bound);
// for K > 1 (VALU bound) a staging ring of two planes, one at radius >= 3
// where K windows of 2R+1 planes fill the budget.
template <int R, int K, int VEC, int WL>
constexpr int prefetch3() {
    constexpr int P = 2 * R + 1;
    if constexpr (K > 1) return R >= 3 ? 1 : 2;
    if constexpr (R > 4) return 1;  // high radius: the z-window alone nears the budget
    if constexpr (VEC == 4 && WL == 32) return P + 3 > 12 ? 3 : 12 - P;  // two rows per wave
    if constexpr (VEC == 4) return P + 4 > 12 ? 4 : 12 - P;  // ring of max(12, P + 4) planes
    return 8 - P > 2 ? 8 - P : 2;                            // ring of max(8, P + 2) planes
}

}  // namespace s3d
}  // namespace star
