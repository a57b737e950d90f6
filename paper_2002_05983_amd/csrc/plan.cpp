// plan.cpp -- kernel configuration and pass schedule of a plan.
#include "plan.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "launch.hpp"
#include "stencil.h"

using namespace star;

namespace {

// Resident wavefronts the 2D kernel aims for: 256 CUs x 4 SIMDs x 4.
constexpr int64_t kTargetWaves2D = 4096;

// Defaults measured on a 16384^2 grid (temporal degree and segment rows):
// the autotuner's picks there.
int default_k2d(int R) {
    switch (R) {
        case 1: return 10;
        case 2: return 6;
        case 3: return 4;
        case 4: return 3;
        case 5: return 3;
        default: return max_k2d(R);
    }
}

int default_ly(const stencil_plan_s *p, int K) {
    const int tx = star2d_tile_x(K, p->radius);
    const int64_t nstrips = (p->nx + tx - 1) / tx;
    // short segments: more wavefronts for the tail of the launch, at the
    // price of re-read wind-up rows (measured best at 64..96 rows)
    int64_t ly = p->radius >= 5 ? 96 : 64;
    // small grids: keep enough wavefronts to fill the chip
    const int64_t want = (p->ny * nstrips + kTargetWaves2D - 1) / kTargetWaves2D;
    ly = std::min<int64_t>(ly, std::max<int64_t>(want, 8 * K * p->radius));
    ly = std::min<int64_t>(ly, p->ny);
    return (int)std::max<int64_t>(ly, 1);
}

// z-segment length: enough workgroups for 2 per CU, without letting the
// 2*K*R wind-up planes exceed a quarter of a segment.
int default_lz(const stencil_plan_s *p) {
    const int W = p->s3_lanes * p->vec;
    const int R = p->radius, K = p->K;
    const bool halo = (int)p->nx > W || p->s3_lanes != 64;
    const int hx = halo ? (K * R + p->vec - 1) / p->vec * p->vec : 0;
    const int64_t tx = halo ? W - 2 * hx : p->nx;
    const int64_t ty = p->s3_rows * (64 / p->s3_lanes) - 2 * K * R;
    const int64_t tiles = ((p->nx + tx - 1) / tx) * ((p->ny + ty - 1) / ty);
    int64_t nseg = (512 + tiles - 1) / tiles;
    int64_t lz = (p->nz + nseg - 1) / nseg;
    lz = std::max<int64_t>(lz, 8 * K * R);
    lz = std::min<int64_t>(lz, p->nz);
    return (int)std::max<int64_t>(lz, 1);
}

// z-segment length of the LDS-free single-step layout: about 4096
// wavefronts (16 per CU), segments of at least 8R planes
// (the 2R wind-up planes are loads only).
int default_lz_rows(const stencil_plan_s *p) {
    const int64_t strips = (p->nx + 255) / 256;
    const int64_t blocks = strips * ((p->ny + p->s3_rpl - 1) / p->s3_rpl);
    const int64_t nseg = std::max<int64_t>(1, (4096 + blocks - 1) / blocks);
    int64_t lz = (p->nz + nseg - 1) / nseg;
    lz = std::max<int64_t>(lz, 8 * p->radius);
    lz = std::min<int64_t>(lz, p->nz);
    return (int)std::max<int64_t>(lz, 1);
}

bool parse_int(const char *s, int *out) {
    char *end = nullptr;
    long v = strtol(s, &end, 10);
    if (end == s || *end != '\0') return false;
    *out = (int)v;
    return true;
}

}  // namespace

static int plan_apply(stencil_plan_s *p, const char *tune);

int plan_configure(stencil_plan_s *p, const char *tune) {
    if (p->storage != STENCIL_F32 && p->ndim != 3)
        return star_set_error(STENCIL_EUNSUPPORTED, "low-precision storage is built for 3D grids");
    if (p->storage != STENCIL_F32 && p->radius > 4)
        return star_set_error(STENCIL_EUNSUPPORTED, "low-precision storage is built for radius 1..4");
    if (tune && *tune) {
        const int rc = plan_apply(p, tune);
        p->tuned_by = "override";
        return rc;
    }
    std::string cached;
    if (tune_cache_lookup(p, cached) && plan_apply(p, cached.c_str()) == STENCIL_OK) {
        p->tuned_by = "cache";
        return STENCIL_OK;
    }
    const int rc = plan_apply(p, nullptr);
    p->tuned_by = "default";
    return rc;
}

static int plan_apply(stencil_plan_s *p, const char *tune) {
    const int R = p->radius;
    if (p->ndim == 2) {
        p->variant = STAR_S2D;
        p->K = default_k2d(R);
        if (p->sym) p->K = std::min(p->K, kMaxKSym2D);
        p->ly = 0;
    } else {
        // defaults measured on a 512^3 grid
        p->variant = STAR_S3D;
        p->K = (p->storage != STENCIL_F32) ? 1 : R == 1 ? 3 : R == 2 ? 2 : 1;
        p->vec = 0;   // chosen below from the grid width
        p->s3_rows = 16;
        p->s3_lanes = 32;
        p->s3_lz = 0;
        p->s3_pair = 0;
        p->s3_rpl = 0;
        p->s3_nbp = 0;
        p->s3_lpr = 64;
        // Above radius 4 the xy-tile kernel's z-queue of 2R+1 planes no
        // longer fits a 1024-thread workgroup's 128 VGPRs (it spills) and 2R
        // of its 32 tile rows are halo; the LDS-free row layout keeps every
        // cell an output cell.
        // From radius 5 on the row layout leads (512^3, two rows per
        // wavefront: 399, 360, 330, 291 GCell/s at R = 5..8 against at most
        // 358, 201, 76, 45 for the tile kernel); unaligned rows take one row
        if (R >= 5 && p->storage == STENCIL_F32) {
            p->s3_rpl = p->nx % 4 == 0 ? 2 : 1;
            p->s3_nbp = 0;
        }
        // At R = 3, 4 the row layout with four rows per wavefront (16-byte
        // rows) beats the tile kernel's single step (512^3: 561 and 528
        // against 522 and 516 GCell/s)
        if ((R == 3 || R == 4) && p->storage == STENCIL_F32 && p->nx % 4 == 0) {
            p->s3_rpl = 4;
            p->s3_nbp = 0;
        }
        // shared coefficients are built into the row layout only
        if (p->sym) {
            p->K = 1;
            p->s3_rpl = 1;
            p->s3_nbp = p->nx % 4 == 0 ? 1 : 0;
        }
    }
    p->ly = (p->ndim == 2) ? 0 : p->ly;
    if (tune && *tune) {
        std::string s(tune);
        size_t pos = 0;
        bool rows_set = false, nbp_set = false;
        while (pos <= s.size()) {
            size_t comma = s.find(',', pos);
            if (comma == std::string::npos) comma = s.size();
            std::string item = s.substr(pos, comma - pos);
            pos = comma + 1;
            if (item.empty()) continue;
            if (item == "naive" && p->storage == STENCIL_F32) {
                p->variant = STAR_NAIVE;
                p->K = 1;
                p->s3_rpl = p->s3_nbp = 0;
                p->s3_lpr = 64;
                continue;
            }
            size_t eq = item.find('=');
            if (eq == std::string::npos)
                return star_set_error(STENCIL_EINVAL, ("bad tune item '" + item + "'").c_str());
            std::string key = item.substr(0, eq), val = item.substr(eq + 1);
            if (key == "nbp" && p->ndim == 3 && (val == "0" || val == "1")) {
                p->s3_nbp = val == "1";
                nbp_set = true;
                p->variant = STAR_S3D;
                continue;
            }
            int v = 0;
            if (!parse_int(val.c_str(), &v) || v < 1)
                return star_set_error(STENCIL_EINVAL, ("bad tune value '" + item + "'").c_str());
            if (key == "k") {
                p->K = v;
                if (v != 1) {  // the row layout is single-step
                    p->s3_rpl = p->s3_nbp = 0;
                    p->s3_lpr = 64;
                }
            } else if (key == "ly" && p->ndim == 2) {
                p->ly = v;
            } else if (key == "lz" && p->ndim == 3) {
                p->s3_lz = v;
                p->variant = STAR_S3D;
            } else if (key == "nw" && p->ndim == 3) {
                p->s3_rows = v;
                p->s3_rpl = p->s3_nbp = 0;  // an xy-tile key selects the xy-tile kernel
                p->s3_lpr = 64;
                p->variant = STAR_S3D;
            } else if (key == "vec" && p->ndim == 3) {
                p->vec = v;
                p->s3_rpl = p->s3_nbp = 0;
                p->s3_lpr = 64;
                p->variant = STAR_S3D;
            } else if (key == "wl" && p->ndim == 3) {
                p->s3_lanes = v;
                p->s3_rpl = p->s3_nbp = 0;
                p->s3_lpr = 64;
                p->variant = STAR_S3D;
            } else if (key == "rows" && p->ndim == 3) {
                p->s3_rpl = v;
                rows_set = true;
                p->variant = STAR_S3D;
            } else if (key == "lpr" && p->ndim == 3) {
                if (v != 64 && v != 16) return star_set_error(STENCIL_EINVAL, "lpr must be 64 or 16");
                p->s3_lpr = v;
                p->variant = STAR_S3D;
            } else if (key == "pair" && p->ndim == 3) {
                if (v != 1) return star_set_error(STENCIL_EINVAL, "pair takes the value 1");
                p->s3_pair = 1;
                p->s3_rpl = p->s3_nbp = 0;
                p->s3_lpr = 64;
                p->variant = STAR_S3D;

            } else {
                return star_set_error(STENCIL_EINVAL, ("unknown tune key '" + key + "'").c_str());
            }
        }
        // 16 lanes per row select the row layout with one row per lane
        // group and no neighbour prefetch, unless rows= / nbp= say otherwise
        if (p->s3_lpr == 16 && p->variant == STAR_S3D) {
            if (!rows_set) p->s3_rpl = 1;
            if (!nbp_set) p->s3_nbp = 0;
        }
    }
    if (p->variant == STAR_S2D) {
        // rows are addressed through one buffer descriptor of nx*4 bytes,
        // whose masked lanes use the offset 2^31
        if (p->nx * 4 >= ((int64_t)1 << 31))
            return star_set_error(STENCIL_EUNSUPPORTED, "2D rows must stay below 2^31 bytes");
        if (p->K < 1 || p->K > max_k2d(R))
            return star_set_error(STENCIL_EINVAL, "2D k must be in 1..16/R (at most 10)");
        if (p->sym && p->K > kMaxKSym2D)
            return star_set_error(STENCIL_EINVAL, "shared coefficients: 2D k must be 1..4");
        if (p->ly == 0) p->ly = default_ly(p, p->K);
        if (p->ly < 1) return star_set_error(STENCIL_EINVAL, "ly must be >= 1");
        p->vec = kVec2D;
        p->tile[0] = star2d_tile_x(p->K, R);
        p->tile[1] = p->ly;
        p->tile[2] = 1;
    } else if (p->variant == STAR_S3D) {
        if (p->nx * p->ny * 4 >= ((int64_t)1 << 31))
            return star_set_error(STENCIL_EUNSUPPORTED, "3D planes must stay below 2^31 bytes");
        if (p->storage != STENCIL_F32) {
            // the low-precision passes are single-step, 4 cells per lane
            if (p->K != 1 || (p->vec != 0 && p->vec != 4) || p->s3_lz % 64 != 0 || p->s3_pair)
                return star_set_error(STENCIL_EINVAL,
                                      "low-precision storage runs k=1, vec=4, lz a multiple of 64, unpaired");
            p->vec = 4;
            if (p->s3_lz == 0) p->s3_lz = 256;  // z-segments of whole 64^3 storage tiles
        }
        if (p->K < 1 || p->K > max_k3d(R))
            return star_set_error(STENCIL_EINVAL, "3D k must be 1..4 for R = 1, 1..3 for R = 2, 3, 1..2 for R = 4..6, 1 above");
        if (p->sym && p->s3_rpl == 0)
            return star_set_error(STENCIL_EINVAL,
                                  "shared coefficients in 3D run the row layout (k=1, rows=1)");
        if (p->s3_rpl > 0 || p->s3_nbp) {
            // LDS-free single-step layout: whole 256-column rows per wavefront
            if (p->s3_rpl == 0) p->s3_rpl = 1;
            if (p->K != 1 || p->storage != STENCIL_F32 || p->s3_pair)
                return star_set_error(STENCIL_EINVAL, "rows= is a single-step FP32 layout (k=1, no pair)");
            if (p->s3_rpl == 3 || p->s3_rpl > 4 || (p->s3_rpl == 4 && (R > 4 || p->s3_nbp)) ||
                (p->s3_rpl == 2 && R > 4 && p->s3_nbp))
                return star_set_error(STENCIL_EINVAL,
                                      "rows must be 1, 2 (nbp=0 above R = 4) or 4 (R <= 4, nbp=0)");
            if (p->sym && p->s3_rpl != 1)
                return star_set_error(STENCIL_EINVAL, "shared coefficients run one row per wavefront");
            if ((p->s3_rpl > 1 || p->s3_nbp) && p->nx % 4 != 0)
                return star_set_error(STENCIL_EINVAL, "rows=2, 4 and nbp=1 need rows of 16 bytes (nx % 4 == 0)");
            if (p->s3_lpr == 16 && (p->s3_rpl != 1 || p->s3_nbp || R > 4 || p->sym))
                return star_set_error(STENCIL_EINVAL,
                                      "lpr=16 runs one row per lane group (rows=1, nbp=0), R <= 4, "
                                      "per-point coefficients");
            if (p->s3_lz == 0) p->s3_lz = default_lz_rows(p);
            if (p->s3_lz < 1) return star_set_error(STENCIL_EINVAL, "lz must be >= 1");
            p->vec = 4;
            p->tile[0] = 4 * p->s3_lpr;
            p->tile[1] = p->s3_rpl * (64 / p->s3_lpr);
            p->tile[2] = p->s3_lz;
            return STENCIL_OK;
        }
        if (p->s3_lanes != 64 && p->s3_lanes != 32)
            return star_set_error(STENCIL_EINVAL, "3D wl must be 64 or 32");
        const int rows = p->s3_rows * (64 / p->s3_lanes);
        if (rows < 2 * p->K * R + 1 || p->s3_rows > 16 || p->s3_rows < 1)
            return star_set_error(STENCIL_EINVAL, "3D nw must be <= 16 with nw*64/wl > 2*k*R");
        const bool al = p->nx % 4 == 0;
        if (p->vec == 0)
            p->vec = (p->s3_lanes == 64 && p->nx > 256 && p->nx <= 512 && vec8_ok(R, p->K, al) &&
                      !p->s3_pair) ? 8 : 4;
        if (p->vec != 4 && !(p->vec == 8 && p->s3_lanes == 64 && vec8_ok(R, p->K, al)))
            return star_set_error(STENCIL_EINVAL, "3D vec must be 4, or 8 for wl=64, aligned k=1, R<=2");
        if (p->s3_pair && (p->K != 1 || p->vec != 4))
            return star_set_error(STENCIL_EINVAL, "pair=1 needs k=1 and vec=4");
        if (p->s3_lz == 0) p->s3_lz = default_lz(p);
        if (p->s3_lz < 1) return star_set_error(STENCIL_EINVAL, "lz must be >= 1");
        const int W = p->s3_lanes * p->vec;
        const bool halo = (int)p->nx > W || p->s3_lanes != 64;
        const int hx = halo ? (p->K * R + p->vec - 1) / p->vec * p->vec : 0;
        p->tile[0] = halo ? W - 2 * hx : (int)p->nx;
        p->tile[1] = rows - 2 * p->K * R;
        p->tile[2] = p->s3_lz;
    } else if (p->variant == STAR_NAIVE) {
        if (p->K != 1) return star_set_error(STENCIL_EINVAL, "naive variant has k = 1");
        p->vec = 1;
        p->tile[0] = p->tile[1] = p->tile[2] = 1;
    }
    return STENCIL_OK;
}

hipError_t plan_enqueue(const stencil_plan_s *p, const float *in, float *out, int64_t steps,
                        hipStream_t stream) {
    if (p->storage != STENCIL_F32) return lowp_enqueue(p, in, out, steps, stream);
    if (steps == 0)
        return hipMemcpyAsync(out, in, (size_t)p->ncells * sizeof(float), hipMemcpyDeviceToDevice,
                              stream);
    std::vector<int> passes;
    plan_pass_schedule(p, steps, passes);
    const int np = (int)passes.size();
    const float *src = in;
    for (int i = 0; i < np; ++i) {
        float *dst = ((np - 1 - i) % 2 == 0) ? out : p->scratch;
        const hipError_t e = plan_launch_pass(p, passes[i], src, dst, stream);
        if (e != hipSuccess) return e;
        src = dst;
    }
    return hipSuccess;
}

void plan_pass_schedule(const stencil_plan_s *p, int64_t steps, std::vector<int> &passes) {
    passes.clear();
    const int K = std::max(1, p->K);
    for (int64_t s = 0; s + K <= steps; s += K) passes.push_back(K);
    if (steps % K) passes.push_back((int)(steps % K));
}

hipError_t plan_launch_pass(const stencil_plan_s *p, int k, const float *src, float *dst,
                            hipStream_t stream) {
    switch (p->variant) {
        case STAR_NAIVE:
            return launch_naive(p->ndim, p->radius, src, dst, (int)p->nx, (int)p->ny, (int)p->nz,
                                p->cf, stream, p->pad, p->sym != 0);
        case STAR_S2D: {
            Star2DArgs a;
            a.src = src;
            a.dst = dst;
            a.nx = (int)p->nx;
            a.ny = (int)p->ny;
            a.K = k;
            // keep the segment length of the full passes for a tail pass
            a.ly = p->ly;
            a.aligned = (p->nx % kVec2D == 0) && ((((uintptr_t)src) | ((uintptr_t)dst)) & 15) == 0;
            a.pad = p->pad;
            a.sym = p->sym != 0;
            a.cf = p->cf;
            switch (p->radius) {
                case 1: return launch_star2d_r1(a, stream);
                case 2: return launch_star2d_r2(a, stream);
                case 3: return launch_star2d_r3(a, stream);
                case 4: return launch_star2d_r4(a, stream);
                case 5: return launch_star2d_r5(a, stream);
                case 6: return launch_star2d_r6(a, stream);
                case 7: return launch_star2d_r7(a, stream);
                case 8: return launch_star2d_r8(a, stream);
            }
            return hipErrorInvalidValue;
        }
        case STAR_S3D: {
            Star3DArgs a;
            a.src = src;
            a.dst = dst;
            a.nx = (int)p->nx;
            a.ny = (int)p->ny;
            a.nz = (int)p->nz;
            a.K = k;
            a.vec = (k == p->K) ? p->vec : 4;  // a tail pass may not fit the wide row
            a.nw = p->s3_rows;
            a.wl = p->s3_lanes;
            a.lz = p->s3_lz;
            a.pair = p->s3_pair != 0 && k == 1;  // a tail pass of a K > 1 plan is not paired
            a.aligned = (p->nx % 4 == 0) && ((((uintptr_t)src) | ((uintptr_t)dst)) & 15) == 0;
            if (a.vec == 8 && !a.aligned) a.vec = 4;
            a.pad = p->pad;
            a.sym = p->sym != 0;
            a.cf = p->cf;
            if (p->s3_rpl > 0 && k == 1) {
                // LDS-free layout; grids not 16-byte aligned take its
                // one-row form without prefetched neighbour rows
                a.rows = a.aligned ? p->s3_rpl : 1;
                a.nbp = a.aligned && p->s3_nbp;
                a.lpr = p->s3_lpr;
                switch (p->radius) {
                    case 1: return launch_star3d_rows_r1(a, stream);
                    case 2: return launch_star3d_rows_r2(a, stream);
                    case 3: return launch_star3d_rows_r3(a, stream);
                    case 4: return launch_star3d_rows_r4(a, stream);
                    case 5: return launch_star3d_rows_r5(a, stream);
                    case 6: return launch_star3d_rows_r6(a, stream);
                    case 7: return launch_star3d_rows_r7(a, stream);
                    case 8: return launch_star3d_rows_r8(a, stream);
                }
                return hipErrorInvalidValue;
            }
            switch (p->radius) {
                case 1: return launch_star3d_r1(a, stream);
                case 2: return launch_star3d_r2(a, stream);
                case 3: return launch_star3d_r3(a, stream);
                case 4: return launch_star3d_r4(a, stream);
                case 5: return launch_star3d_r5(a, stream);
                case 6: return launch_star3d_r6(a, stream);
                case 7: return launch_star3d_r7(a, stream);
                case 8: return launch_star3d_r8(a, stream);
            }
            return hipErrorInvalidValue;
        }
        default:
            return hipErrorInvalidValue;
    }
}

std::string plan_describe(const stencil_plan_s *p) {
    std::string s = plan_describe_config(p);
    if (p->pad) s += " boundary=padded";
    if (p->sym) s += " coeffs=shared";
    return s;
}

std::string plan_describe_config(const stencil_plan_s *p) {
    char buf[256];
    const char *v = p->variant == STAR_NAIVE ? "naive" : p->variant == STAR_S2D ? "s2d" : "s3d";
    if (p->variant == STAR_S3D && p->s3_rpl > 0)
        snprintf(buf, sizeof buf, "variant=s3d ndim=3 R=%d K=1 layout=rows rows=%d nbp=%d lz=%d%s by=%s",
                 p->radius, p->s3_rpl, p->s3_nbp, p->s3_lz, p->s3_lpr == 16 ? " lpr=16" : "",
                 p->tuned_by.c_str());
    else if (p->variant == STAR_S3D)
        snprintf(buf, sizeof buf,
                 "variant=%s ndim=3 R=%d K=%d tile=%dx%dx%d vec=%d wl=%d nw=%d lz=%d%s%s by=%s",
                 p->storage == STENCIL_F32 ? "s3d"
                 : p->storage == STENCIL_F16 ? "s3d-f16"
                 : p->storage == STENCIL_BF16 ? "s3d-bf16"
                 : p->storage == STENCIL_F16_SCALED ? "s3d-f16-scaled" : "s3d-bf16-scaled",
                 p->radius, p->K, p->tile[0], p->tile[1], p->tile[2], p->vec, p->s3_lanes,
                 p->s3_rows, p->s3_lz, p->s3_pair ? " pair=1" : "",
                 p->storage == STENCIL_F32 ? ""
                 : (" m=" + std::to_string(p->anchor_m)).c_str(),
                 p->tuned_by.c_str());
    else
        snprintf(buf, sizeof buf, "variant=%s ndim=%d R=%d K=%d tile=%dx%dx%d vec=%d ly=%d by=%s", v,
                 p->ndim, p->radius, p->K, p->tile[0], p->tile[1], p->tile[2], p->vec, p->ly,
                 p->tuned_by.c_str());
    return buf;
}

void plan_release_extra(stencil_plan_s *p) { lowp_release(p); }
