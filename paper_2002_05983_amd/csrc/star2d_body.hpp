// star2d_body.hpp -- 2D star stencil, x-strip per wavefront, y streamed, K fused steps.
//
// The per-wavefront body shared by the single-grid kernel and the batched
// work-list kernel.
//
// Method (Sec. III.A of the paper: 1.5D spatial blocking -- block x, stream
// y -- combined with temporal blocking by a chain of K stages and
// overlapped halos, Eq. (2)):
//   * One wavefront owns a strip of 64 lanes x 4 cells = 256 columns: a
//     TX-column output tile plus a halo of H = roundup(K*R, 4) columns per
//     side.  Each lane holds 4 consecutive cells of a row; rows are read and
//     written with one 128-bit access per lane.
//   * The wavefront streams rows y0-K*R .. y1-1+K*R of its y-segment.  Stage
//     s (1..K) applies one time step and runs R rows behind stage s-1, like
//     the paper's PE chain; it starts once its first needed row
//     (y0-(K-s)*R) is due, 2*s*R rows into the stream.  Each stage keeps the last 2R+1 rows of its input
//     in a register queue: the y-neighbours.  The x-neighbours of the
//     queue's centre row come from the lane's own registers and, across the
//     lane boundary, from the adjacent lanes through DPP wave shifts (fused
//     into the FMA that uses them in the interior form).  Only
//     the K-th stage is written back, so one pass moves 8 bytes per cell for
//     K steps.
//   * Halo cells are recomputed by neighbouring strips instead of exchanged
//     (overlapped blocking); the invalid region grows R columns per stage
//     from each strip edge and never reaches the output tile.
//   * Clamp boundary (Sec. III.B), applied to every stage's field: rows
//     above the grid are filled with the stage's row 0 when it is produced,
//     rows below take the stage's row ny-1, and columns outside [0, nx) are
//     overwritten with the border column of the same stage and row.
//   * Each cell is c_C*f_C followed by one FMA per neighbour in coefficient
//     order (W, E, S, N for i = 1..R), the library-wide operation order.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace star {
namespace s2d {

constexpr int VEC = kVec2D;

// Cells of one row of one stage.  q is a circular buffer of rows of the
// stage's input (NS slots); CS is the slot of the centre row (compile-time).
// EDGE: the strip may hold the grid's border, so the lanes at the ends of
// the wavefront take their own outermost cell as the missing neighbour;
// otherwise those lanes hold halo columns whose values never reach the
// output and the shifts fill them with zero.
// SYM: shared coefficients, one per axis and distance (cf holds c_C, then
// c_x,i, c_y,i for i = 1..R): per distance, one FMA with the rounded sum of
// the W and E cells, then one with the sum of the S and N cells.
// Fused-shift form: the interior form with per-point coefficients, where
// the lanes at the wavefront's ends hold halo columns (their values never
// reach the output): an FMA whose x-neighbour lies in the adjacent lane
// takes it through the wave shift of its own operand (fma_shifted), which
// saves the separate shift of each of the 2R border values of a row; a
// neighbour two lanes away (distances 5..8) moves one lane by a plain
// shift first.
template <int R, bool EDGE, bool SYM>
constexpr bool star2d_fused_shift() { return !EDGE && !SYM && R <= 2 * VEC; }

template <int R, int NS, int CS, bool EDGE, bool SYM = false>
__device__ __forceinline__ void star2d_row(const float (&q)[NS][VEC], const Coefs &cf,
                                           const XCoefV<R> &xv, float (&res)[VEC]) {
    static_assert(R <= 2 * VEC, "x-neighbours come from the lanes at most two away");
    if constexpr (star2d_fused_shift<R, EDGE, SYM>()) {
        // distance by distance over the lane's cells: each cell's FMAs keep
        // their order (W, E, S, N per distance); the FMAs of one distance
        // and side that reach across the lane boundary form one fused block
        float acc[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e] = cf.c[0] * q[CS][e];
        static_for<1, R + 1>([&](auto ic) STAR_INLINE {
            constexpr int i = decltype(ic)::value;
            // cells whose neighbour at distance i lies in another lane: the
            // first (W) or last (E) NX of them; at i > VEC two lanes away for
            // some, whose value first moves one lane by a plain shift
            constexpr int NX = i < VEC ? i : VEC;
            // W terms of the cells e >= i (own lane), then one fused block
            // with the W terms of the first NX cells (lanes below) and the
            // E terms of the last NX (lanes above), then the E terms of the
            // cells e < VEC - i (own lane): each cell keeps W before E
#pragma unroll
            for (int e = i; e < VEC; ++e)
                acc[e] = __builtin_fmaf(cf.c[coef_index<2>(kW, i)], q[CS][e - i], acc[e]);
            {
                float vw[NX], ve[NX];
#pragma unroll
                for (int e = 0; e < NX; ++e) {
                    const int off = e - i;  // column offset from the lane's base, < 0
                    vw[e] = (off >= -VEC) ? q[CS][(VEC + off) & (VEC - 1)]
                                          : from_lower_lane_or_zero(q[CS][(2 * VEC + off) & (VEC - 1)]);
                }
#pragma unroll
                for (int k = 0; k < NX; ++k) {
                    const int off = k + i - NX;  // element in the lane above, >= 0
                    ve[k] = (off < VEC) ? q[CS][off & (VEC - 1)]
                                        : from_upper_lane_or_zero(q[CS][(off - VEC) & (VEC - 1)]);
                }
                fma_shifted_we<i>(acc, xv.w[i], vw, xv.e[i], ve);
            }
#pragma unroll
            for (int e = 0; e < VEC - i; ++e)
                acc[e] = __builtin_fmaf(cf.c[coef_index<2>(kE, i)], q[CS][e + i], acc[e]);
#pragma unroll
            for (int e = 0; e < VEC; ++e) {
                acc[e] = __builtin_fmaf(cf.c[coef_index<2>(kS, i)], q[(CS - i + NS) % NS][e], acc[e]);
                acc[e] = __builtin_fmaf(cf.c[coef_index<2>(kN, i)], q[(CS + i) % NS][e], acc[e]);
            }
        });
#pragma unroll
        for (int e = 0; e < VEC; ++e) res[e] = acc[e];
        return;
    }
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
        } else {  // two lanes away
            left[k] = lower(lower(q[CS][2 * VEC - k]));
            right[k] = upper(upper(q[CS][k - VEC - 1]));
        }
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
        float acc = cf.c[0] * q[CS][e];
#pragma unroll
        for (int i = 1; i <= R; ++i) {
            const float w = (e - i >= 0) ? q[CS][e - i] : left[i - e];
            const float ea = (e + i < VEC) ? q[CS][e + i] : right[e + i - VEC + 1];
            const float s = q[(CS - i + NS) % NS][e];
            const float n = q[(CS + i) % NS][e];
            if constexpr (SYM) {
                acc = __builtin_fmaf(cf.c[1 + 2 * (i - 1)], w + ea, acc);
                acc = __builtin_fmaf(cf.c[2 + 2 * (i - 1)], s + n, acc);
            } else {
                acc = __builtin_fmaf(cf.c[coef_index<2>(kW, i)], w, acc);
                acc = __builtin_fmaf(cf.c[coef_index<2>(kE, i)], ea, acc);
                acc = __builtin_fmaf(cf.c[coef_index<2>(kS, i)], s, acc);
                acc = __builtin_fmaf(cf.c[coef_index<2>(kN, i)], n, acc);
            }
        }
        res[e] = acc;
    }
}

// One wavefront's work: strip `strip` (TX output columns) of y-segment `seg`
// (ly output rows) of one grid.  Wave-level: no barriers, no LDS.  Every
// argument is wave-uniform.  EDGE = false is the interior form: the strip's
// columns and every row its stages touch lie inside the grid
// (star2d_interior), so no clamp is ever applied and the border code is
// left out; for such a strip it computes the same bits as the general form.
// pad > 0: padded-halo boundary (Sec. IV.B): the grid is the padded array
// and its frame of `pad` cells is fixed, so in the general form every stage
// gives a frame cell its own (unchanged) value; the interior form never
// holds a frame cell among the cells that reach the output (the interior
// test is shrunk by the frame).
template <int R, int K, int D, bool ALIGNED, bool EDGE = true, bool SYM = false>
__device__ __forceinline__ void star2d_body(const float *__restrict__ src, float *__restrict__ dst,
                                            int nx, int ny, int ly, int strip, int seg,
                                            const Coefs &cf, int pad = 0) {
    constexpr int P = 2 * R + 1;  // rows a stage keeps: its y-window
    constexpr int NQ = P + D;     // input ring: y-window plus D rows in flight
    // stage s >= 2 keeps its window in slot (ring slot mod P), which follows
    // the row index only when P divides the ring length
    static_assert(K == 1 || D % P == 0, "prefetch distance must be a multiple of the y-window");
    constexpr int H = star2d_halo(K, R);
    constexpr int TX = star2d_tile_x(K, R);

    const int lane = threadIdx.x & 63;
    const int xs = strip * TX - H;  // first column held by lane 0
    const int col0 = xs + lane * VEC;
    const int y0 = seg * ly;
    const int y1 = min(y0 + ly, ny);
    const int jstart = y0 - K * R;
    const int niter = (y1 - y0) + 2 * K * R;
    const int jlast = jstart + niter - 1;
    const bool left_edge = xs < 0;
    const bool right_edge = xs + 64 * VEC > nx;
    // the wavefront holds a column of the padded-halo frame
    const bool frame_cols = xs < pad || xs + 64 * VEC > nx - pad;
    const int out_lo = max(xs + H, 0);
    const int out_hi = min(xs + H + TX, nx);

    // Clamp in x: cells left of column 0 take column 0, cells right of
    // column nx-1 take column nx-1 (of the same row and stage).
    auto xfix = [&](float (&v)[VEC]) STAR_INLINE {
        if constexpr (!EDGE) return;
        if (left_edge) {
            const int l0 = (-xs) / VEC;  // lane whose element 0 is column 0
            const float b = lane_value(v[0], l0);
            if (lane < l0) {
#pragma unroll
                for (int e = 0; e < VEC; ++e) v[e] = b;
            }
        }
        if (right_edge) {
            const int off = nx - 1 - xs;
            const int lr = off / VEC, er = off % VEC;
            float t = v[0];
#pragma unroll
            for (int e = 1; e < VEC; ++e) t = (er == e) ? v[e] : t;
            const float b = lane_value(t, lr);
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[e] = (col0 + e >= nx) ? b : v[e];
        }
    };

    // Issues the load of input row j (clamped to the grid in y) into v.
    // Rows past the segment's last one are never needed; they are re-read
    // as the last row.  The x-clamp of a loaded row is applied when the row
    // enters stage 1 (consume_row), so no load is waited for early.
    auto load_row = [&](int j, float (&v)[VEC]) STAR_INLINE {
        const float *row = src + (size_t)(EDGE ? clampi(min(j, jlast), ny) : min(j, jlast)) * (size_t)nx;
        if constexpr (ALIGNED) {
            const int c = EDGE ? min(max(col0, 0), nx - VEC) : col0;
            const float4 t = *reinterpret_cast<const float4 *>(row + c);
            v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
        } else {
#pragma unroll
            for (int e = 0; e < VEC; ++e) v[e] = row[EDGE ? clampi(col0 + e, nx) : col0 + e];
        }
    };

    XCoefV<R> xv;
    if constexpr (star2d_fused_shift<R, EDGE, SYM>()) {
#pragma unroll
        for (int i = 1; i <= R; ++i) {
            xv.w[i] = vgpr_copy(cf.c[coef_index<2>(kW, i)]);
            xv.e[i] = vgpr_copy(cf.c[coef_index<2>(kE, i)]);
        }
    }

    // q0: ring of NQ input rows, loaded straight into their slots.
    // q[s-1] (s = 2..K): last P rows of the stage-(s-1) field.
    float q0[NQ][VEC];
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

    constexpr int DIST = D;  // prefetch distance in rows
    static_for<0, DIST>([&](auto phc) STAR_INLINE {
        constexpr int PH = decltype(phc)::value;
        load_row(jstart + PH, q0[PH]);
    });

    // One streamed row: iteration n, ring slot PH = n mod NQ.
    auto step_row = [&](auto phc, int n) STAR_INLINE {
        constexpr int PH = decltype(phc)::value;
        const int j = jstart + n;  // row entering stage 1
        load_row(j + DIST, q0[(PH + DIST) % NQ]);
        if constexpr (ALIGNED) xfix(q0[PH]);

        static_for<1, K + 1>([&](auto sc) STAR_INLINE {
            constexpr int S = decltype(sc)::value;
            // Stage S first produces a row that an output depends on at
            // iteration 2*S*R; before that its window still holds wind-up
            // rows and nothing reads what it would produce.
            if (n < 2 * S * R) return;
            const int r = j - S * R;  // row produced by stage S
            float res[VEC];
            if constexpr (S == 1)
                star2d_row<R, NQ, (PH - R + NQ) % NQ, EDGE, SYM>(q0, cf, xv, res);
            else
                star2d_row<R, P, (PH % P - R + P) % P, EDGE, SYM>(q[S - 2], cf, xv, res);
            if constexpr (EDGE) {
                // the fixed frame of the padded array keeps its values: a
                // frame cell takes its centre (this stage's input); the
                // per-cell select only where the row or the wavefront's
                // columns touch the frame (wave-uniform test)
                const bool frame_row = r < pad || r >= ny - pad;
                if (pad > 0 && (frame_row || frame_cols)) {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        float ctr;
                        if constexpr (S == 1)
                            ctr = q0[(PH - R + NQ) % NQ][e];
                        else
                            ctr = q[S - 2][(PH % P - R + P) % P][e];
                        const int c = col0 + e;
                        res[e] = (frame_row || c < pad || c >= nx - pad) ? ctr : res[e];
                    }
                }
            }
            if constexpr (S < K) {
                constexpr int W = PH % P;  // slot of this row in the stage's window
                if constexpr (EDGE) {
                    if (r >= ny) {
#pragma unroll
                        for (int e = 0; e < VEC; ++e) res[e] = q[S - 1][(W + P - 1) % P][e];
                    } else {
                        xfix(res);
                    }
                }
#pragma unroll
                for (int e = 0; e < VEC; ++e) q[S - 1][W][e] = res[e];
                if constexpr (EDGE) {
                    if (r == 0) {
                        static_for<1, R + 1>([&](auto mc) STAR_INLINE {
                            constexpr int MM = decltype(mc)::value;
#pragma unroll
                            for (int e = 0; e < VEC; ++e) q[S - 1][(W - MM + P) % P][e] = res[e];
                        });
                    }
                }
            } else {
                // Stage K: write row r.  The store is issued on every row;
                // rows of the wind-up and lanes outside the output tile get
                // an out-of-range offset and write nothing.
                const bool row_ok = r >= y0 && r < y1;
                const auto rs = buffer_rsrc(dst + (size_t)clampi(r, ny) * (size_t)nx, nx * 4);
                if constexpr (ALIGNED) {
                    const bool ok = row_ok && col0 >= out_lo && col0 + VEC <= out_hi;
                    buffer_store4<kStoreNT>(rs, ok ? col0 * 4 : kOutOfRange, res[0], res[1], res[2], res[3]);
                } else {
#pragma unroll
                    for (int e = 0; e < VEC; ++e) {
                        const int c = col0 + e;
                        const bool ok = row_ok && c >= out_lo && c < out_hi;
                        buffer_store1<kStoreNT>(rs, ok ? c * 4 : kOutOfRange, res[e]);
                    }
                }
            }
        });
    };

    int n0 = 0;
    for (; n0 + NQ <= niter; n0 += NQ) {
        static_for<0, NQ>([&](auto phc) STAR_INLINE { step_row(phc, n0 + decltype(phc)::value); });
    }
    static_for<0, NQ>([&](auto phc) STAR_INLINE {
        if (n0 + decltype(phc)::value < niter) step_row(phc, n0 + decltype(phc)::value);
    });
}

// True when strip `strip` of segment `seg` needs no clamp at any stage: its
// 64*VEC columns lie inside the grid, and rows y0-2KR .. y1-1+KR (the rows
// its stages read and produce) do too.  With a padded-halo frame of `pad`
// cells the same must hold inside the frame, so that no frame cell is
// updated.
template <int R, int K>
__device__ __forceinline__ bool star2d_interior(int nx, int ny, int ly, int strip, int seg,
                                                int pad = 0) {
    const int xs = strip * star2d_tile_x(K, R) - star2d_halo(K, R);
    const int y0 = seg * ly;
    const int y1 = min(y0 + ly, ny);
    return xs >= pad && xs + 64 * VEC <= nx - pad && y0 > 2 * K * R + pad &&
           y1 + K * R <= ny - pad;
}

// Rows in flight per wavefront: two y-windows for the memory-bound small-K
// passes and for R = 1, K = 8 (measured on 16384^2: +2 %; at K = 5..7 the
// extra registers cost a wave per SIMD and 2-4 %), one otherwise, and 8
// rows (8 KiB per wavefront) for single-step passes of R >= 5, where a
// whole window would cost more registers than the latency needs.  With
// K > 1 it must be a multiple of the window (the stages' window slots are
// derived from the input-ring slot).
template <int R, int K>
constexpr int prefetch_rows() {
    return (K * R <= 2 || (R == 1 && K == 8)) ? 2 * (2 * R + 1) : (K == 1 && R >= 5) ? 8 : 2 * R + 1;
}

}  // namespace s2d
}  // namespace star
