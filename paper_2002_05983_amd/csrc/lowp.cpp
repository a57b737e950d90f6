// lowp.cpp -- host schedule of the precision form (anchored low-precision delta).
//
// State: FP32 anchor A (the plan's scratch) and a delta D stored as 16-bit
// codes with one power-of-two scale per 64^3 tile, F = A + D.  Per window of
// m steps (one FP32 anchor per window):
//   G32 = S A - A            FP32 pass, records max|G32| per tile
//   eG  from max|G32|;  G16 = encode(G32)
//   D   = G16                (the delta after the window's first step)
//   m-1 times:  e' from the bound  s1*max_{27 nbr tiles}|D| + max|G32|
//               D = encode(S decode(D) + decode(G16)), records max|value|
//   A   = A + decode(D)      (the last window writes `out` instead)
// Maxima are taken before rounding to codes; s1 = sum |c| bounds one step's
// growth, so codes stay within +-2^14 (1 + 2^-11), far below FP16's limit.
//
// The scaled-state form (STENCIL_F16_SCALED / STENCIL_BF16_SCALED) keeps the
// state itself as codes between FP32 anchor steps.  Per window of m steps:
//   eQ  from max|A| per tile;  Q = encode(A)
//   m-1 times:  e' from the bound  s1*max_{27 nbr tiles}|Q|
//               Q = encode(S decode(Q)), records max|value| before rounding
//   A   = S decode(Q)        one FP32 step (the anchor; the last window
//                            writes `out`)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "lowp.hpp"
#include "plan.hpp"
#include "stencil.h"

using namespace star;

struct LowpState {
    int tnx = 0, tny = 0, tnz = 0, ntiles = 0;
    uint16_t *d16[2] = {nullptr, nullptr};
    uint16_t *g16 = nullptr;
    int *e_d[2] = {nullptr, nullptr};
    int *e_g = nullptr;
    unsigned *max_d[2] = {nullptr, nullptr};
    unsigned *max_g32 = nullptr;
    unsigned *max_g16 = nullptr;
    double s1 = 0.0;
};

namespace {

hipError_t launch_pass(const stencil_plan_s *p, const LowpArgs &a, int mode, hipStream_t s) {
    switch (p->radius) {
        case 1: return launch_lowp3d_r1(a, mode, s);
        case 2: return launch_lowp3d_r2(a, mode, s);
        case 3: return launch_lowp3d_r3(a, mode, s);
        case 4: return launch_lowp3d_r4(a, mode, s);
    }
    return hipErrorInvalidValue;
}

#define LP_TRY(x)                               \
    do {                                        \
        const hipError_t e__ = (x);             \
        if (e__ != hipSuccess) return e__;      \
    } while (0)

}  // namespace

int lowp_allocate(stencil_plan_s *p) {
    if (p->ndim != 3) return star_set_error(STENCIL_EUNSUPPORTED, "low-precision storage is built for 3D grids");
    if (p->nx % 4 != 0 || p->nx < 4)
        return star_set_error(STENCIL_EUNSUPPORTED, "low-precision storage needs nx % 4 == 0");
    auto *s = new (std::nothrow) LowpState();
    if (!s) return star_set_error(STENCIL_ENOMEM, "host allocation failed");
    s->tnx = (int)((p->nx + 63) >> kTileShift);
    s->tny = (int)((p->ny + 63) >> kTileShift);
    s->tnz = (int)((p->nz + 63) >> kTileShift);
    s->ntiles = s->tnx * s->tny * s->tnz;
    for (int k = 0; k < p->npts; ++k) s->s1 += std::fabs((double)p->cf.c[k]);
    const size_t codes = (size_t)p->ncells * sizeof(uint16_t);
    const size_t tab = (size_t)s->ntiles * sizeof(int);
    bool ok = hipMalloc(&s->d16[0], codes) == hipSuccess && hipMalloc(&s->d16[1], codes) == hipSuccess &&
              hipMalloc(&s->g16, codes) == hipSuccess && hipMalloc(&s->e_d[0], tab) == hipSuccess &&
              hipMalloc(&s->e_d[1], tab) == hipSuccess && hipMalloc(&s->e_g, tab) == hipSuccess &&
              hipMalloc(&s->max_d[0], tab) == hipSuccess && hipMalloc(&s->max_d[1], tab) == hipSuccess &&
              hipMalloc(&s->max_g32, tab) == hipSuccess && hipMalloc(&s->max_g16, tab) == hipSuccess;
    p->lowp = s;
    if (!ok) {
        (void)hipGetLastError();
        return star_set_error(STENCIL_ENOMEM, "device allocation of the low-precision state failed");
    }
    return STENCIL_OK;
}

void lowp_release(stencil_plan_s *p) {
    LowpState *s = p->lowp;
    if (!s) return;
    for (void *q : {(void *)s->d16[0], (void *)s->d16[1], (void *)s->g16, (void *)s->e_d[0],
                    (void *)s->e_d[1], (void *)s->e_g, (void *)s->max_d[0], (void *)s->max_d[1],
                    (void *)s->max_g32, (void *)s->max_g16})
        if (q) (void)hipFree(q);
    delete s;
    p->lowp = nullptr;
}

namespace {

// The scaled-state schedule (see the top of this file).
hipError_t scaled_enqueue(const stencil_plan_s *p, const float *in, float *out, int64_t steps,
                          hipStream_t st) {
    LowpState *s = p->lowp;
    const int codec = p->storage == STENCIL_F16_SCALED ? kCodecF16 : kCodecBF16;
    const int nx = (int)p->nx, ny = (int)p->ny, nz = (int)p->nz;
    float *A = p->scratch;
    LowpArgs a{};
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.nw = p->s3_rows;
    a.wl = p->s3_lanes;
    a.lz = p->s3_lz;
    a.tnx = s->tnx;
    a.tny = s->tny;
    a.tnz = s->tnz;
    a.cf = p->cf;
    // the bound has no G term: its table stays zero
    LP_TRY(lowp_fill_u32(s->max_g16, s->ntiles, 0u, st));
    // FP32 state at the window start (read with 16-byte vector loads)
    const float *cur = in;
    if ((uintptr_t)in & 15) {
        LP_TRY(hipMemcpyAsync(A, in, (size_t)p->ncells * sizeof(float), hipMemcpyDeviceToDevice, st));
        cur = A;
    }
    int64_t t = 0;
    while (t < steps) {
        const int64_t w = std::min<int64_t>(p->anchor_m, steps - t);
        // exact scales from max|state|, then Q = encode(state)
        LP_TRY(lowp_fill_u32(s->max_g32, s->ntiles, 0u, st));
        LP_TRY(lowp_tile_max(cur, s->max_g32, nx, ny, nz, s->tnx, s->tny, st));
        LP_TRY(lowp_exponents_from_max(s->max_g32, s->ntiles, s->e_g, st));
        LP_TRY(lowp_encode(codec, cur, s->e_g, s->g16, nx, ny, nz, s->tnx, s->tny, st));
        const uint16_t *q = s->g16;
        const int *e_q = s->e_g;
        const unsigned *max_q = s->max_g32;
        for (int64_t j = 1; j < w; ++j) {
            const int o = (int)(j & 1);
            LP_TRY(lowp_exponents_from_bound(max_q, s->max_g16, s->s1, s->tnx, s->tny, s->tnz,
                                             s->e_d[o], st));
            unsigned *mo = s->max_d[o];  // not the table being read
            LP_TRY(lowp_fill_u32(mo, s->ntiles, 0u, st));
            a.d_in = q;
            a.e_in = e_q;
            a.g = q;  // unused (no G term)
            a.e_g = e_q;
            a.d_out = s->d16[o];
            a.e_out = s->e_d[o];
            a.max_out = mo;
            LP_TRY(launch_pass(p, a, kScaledPass + codec, st));
            q = s->d16[o];
            e_q = s->e_d[o];
            max_q = mo;
        }
        t += w;
        // anchor: one FP32 step from the decoded state
        float *dst = t < steps ? A : out;
        float *tmp = t < steps ? out : A;
        LP_TRY(lowp_add_decoded(codec, nullptr, q, e_q, tmp, nx, ny, nz, s->tnx, s->tny, st));
        LP_TRY(plan_launch_pass(p, 1, tmp, dst, st));
        cur = A;
    }
    return hipSuccess;
}

}  // namespace

hipError_t lowp_enqueue(const stencil_plan_s *p, const float *in, float *out, int64_t steps,
                        hipStream_t st) {
    const size_t bytes = (size_t)p->ncells * sizeof(float);
    if (steps == 0) return hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, st);
    if (p->storage == STENCIL_F16_SCALED || p->storage == STENCIL_BF16_SCALED)
        return scaled_enqueue(p, in, out, steps, st);
    LowpState *s = p->lowp;
    const int codec = p->storage;  // STENCIL_F16 == kCodecF16, STENCIL_BF16 == kCodecBF16
    const int nx = (int)p->nx, ny = (int)p->ny, nz = (int)p->nz;
    float *A = p->scratch;
    LP_TRY(hipMemcpyAsync(A, in, bytes, hipMemcpyDeviceToDevice, st));

    LowpArgs a{};
    a.nx = nx;
    a.ny = ny;
    a.nz = nz;
    a.nw = p->s3_rows;
    a.wl = p->s3_lanes;
    a.lz = p->s3_lz;
    a.tnx = s->tnx;
    a.tny = s->tny;
    a.tnz = s->tnz;
    a.cf = p->cf;
    int64_t t = 0;
    while (t < steps) {
        const int64_t w = std::min<int64_t>(p->anchor_m, steps - t);
        // G = S A - A, staged in FP32 in `out`, then encoded with exact tile scales
        LP_TRY(lowp_fill_u32(s->max_g32, s->ntiles, 0u, st));
        a.a_in = A;
        a.g_out = out;
        a.max_out = s->max_g32;
        LP_TRY(launch_pass(p, a, 0, st));
        LP_TRY(lowp_exponents_from_max(s->max_g32, s->ntiles, s->e_g, st));
        LP_TRY(lowp_encode(codec, out, s->e_g, s->g16, nx, ny, nz, s->tnx, s->tny, st));
        // D after the first step of the window is G itself
        const uint16_t *d = s->g16;
        const int *e_d = s->e_g;
        const unsigned *max_d = s->max_g32;
        for (int64_t j = 1; j < w; ++j) {
            const int o = (int)(j & 1);
            LP_TRY(lowp_exponents_from_bound(max_d, s->max_g32, s->s1, s->tnx, s->tny, s->tnz,
                                             s->e_d[o], st));
            LP_TRY(lowp_fill_u32(s->max_d[o], s->ntiles, 0u, st));
            a.d_in = d;
            a.e_in = e_d;
            a.g = s->g16;
            a.e_g = s->e_g;
            a.d_out = s->d16[o];
            a.e_out = s->e_d[o];
            a.max_out = s->max_d[o];
            LP_TRY(launch_pass(p, a, codec, st));
            d = s->d16[o];
            e_d = s->e_d[o];
            max_d = s->max_d[o];
        }
        t += w;
        // re-anchor in FP32 (the last window writes the result)
        LP_TRY(lowp_add_decoded(codec, A, d, e_d, t < steps ? A : out, nx, ny, nz, s->tnx, s->tny,
                                st));
    }
    return hipSuccess;
}
