// model.cpp -- analytic throughput model of the streaming kernels.
//
// The paper sizes its FPGA design with a performance model before building
// the top candidates (Sec. V.A).  This is the GPU counterpart for the kernels
// here: a pass of K fused steps is bounded by the largest of
//   HBM     bytes the pass must move / effective bandwidth;
//   VALU    wavefront instructions / (CUs x SIMDs), 4 cycles per wave64
//           instruction on a 16-lane SIMD; in 2D counted in rounds of the
//           wavefronts each SIMD holds (estimated from the kernel's
//           registers), a SIMD with a lone wavefront issuing at half rate;
//   stream  (3D) the sequential path: the per-plane critical path of a
//           workgroup -- its VALU issue, LDS write, barrier, LDS reads --
//           times the planes each CU streams one after the other;
// plus a launch cost.  Instruction counts are written from the kernels'
// structure (4 cells per lane, one FMA per point, 2R lane shifts per row and
// stage, fused into the FMAs of the 2D interior form for R <= 4) with a
// per-row overhead constant; the constants are fitted to this
// GPU's measurements and the fit is reported as model accuracy.
#include <algorithm>
#include <cmath>

#include "launch.hpp"
#include "plan.hpp"
#include "stencil.h"

using namespace star;

namespace {

constexpr double kCUs = 256.0;
constexpr double kSimdPerCU = 4.0;
constexpr double kClock = 2.4e9;             // Hz
constexpr double kCyclesPerWaveInstr = 4.0;  // wave64 on a 16-lane SIMD
// Fitted to the autotuner's measurements on MI355X (every candidate of 23
// problems: 2D 16384^2 at R = 1..8 and 4096^2 at R = 1..4, 3D 512^3 at
// R = 1..8, 768^3, 256^3 and 192x256x320) by a coordinate grid search
// minimising the median |log(predicted / measured)| plus the shortfall of
// the model's pick from the measured best:
constexpr double kHbmEff2D = 5.0e12, kHbmEff3D = 5.0e12;  // B/s reached by the passes
// s per pass: launch, plus (2D) the ramp-up and drain of the last wavefronts
constexpr double kLaunch2D = 30e-6, kLaunch3D = 10e-6;
// instructions per wavefront row and stage beyond the FMAs and lane shifts
// (clamps, register moves, index arithmetic, issue stalls), and per streamed row
constexpr double kRowStage2D = 5.0, kRow2D = 2.0;
// Measured in 2D, not derived: the rate falls with the segment length at
// high K (16384^2, R = 1, K = 8: 4263 GCell/s at ly = 64, 2987 at ly = 384;
// flat at K = 1), fitted as a factor 1 + kLyPenalty (ly/64 - 1) K/8 on the
// pass time.
constexpr double kLyPenalty = 0.1;
constexpr double kRowStage3D = 25.0, kRow3D = 24.0, kLoadOnly3D = 30.0;
// a wavefront alone on its SIMD issues one VALU instruction per kLoneIssue x
// 4 cycles (dependent FMA chains); kLoneIssue of them keep the SIMD busy
constexpr double kLoneIssue = 2.0;
// per-plane critical path of a 3D workgroup beyond its VALU issue time
// (LDS write, barrier, LDS reads), cycles
constexpr double kPlaneLatency3D = 300.0;
// the xy-tile kernel spills above radius 4 (its z-queue of 2R+1 planes
// outgrows 128 VGPRs): issue time x (1 + kSpill (KR - 4)^2), and fused
// steps from radius 4 on x (1 + kSpillK (K - 1) R)
constexpr double kSpill = 0.5, kSpillK = 0.1;
// the row layout's neighbour rows that miss L2: kMissSlope (R - 1), at most kMissMax
constexpr double kMissSlope = 0.1, kMissMax = 0.2;

struct Pass {
    double t_hbm, t_valu, t_plane;
    double scale = 1.0;  // empirical factor on the pass time
};

// Rows in flight per 2D wavefront (the rule of prefetch_rows in
// star2d_body.hpp) and the resulting waves per SIMD: 4 floats per row of
// the input ring and of the K-1 stage windows, ~24 registers besides.
int prefetch_2d(int R, int K) {
    if (K * R <= 2 || (R == 1 && K == 8)) return 2 * (2 * R + 1);
    if (K == 1 && R >= 5) return 8;
    return 2 * R + 1;
}
int waves_per_simd_2d(int R, int K) {
    const int P = 2 * R + 1;
    const int vgprs = (kVec2D * (P + prefetch_2d(R, K) + (K - 1) * P) + 24 + 7) / 8 * 8;
    return std::max(1, std::min(8, 512 / vgprs));
}

// Issue time of `waves` wavefronts of `per_wave` VALU instructions on the
// 1024 SIMDs, at most `occ` at a time on each: full rounds, then the rest
// spread evenly; a SIMD holding w < kLoneIssue wavefronts issues w
// instructions per kLoneIssue x 4 cycles.
double simd_time(double waves, double per_wave, int occ) {
    const double simds = kCUs * kSimdPerCU, slots = simds * occ;
    const double full = std::floor(waves / slots), rest = waves - full * slots;
    double t = full * occ * per_wave * std::max(1.0, kLoneIssue / occ);
    if (rest > 0) {
        const double w = std::ceil(rest / simds);
        t += w * per_wave * std::max(1.0, kLoneIssue / w);
    }
    return t * kCyclesPerWaveInstr / kClock;
}

Pass model_2d(const stencil_plan_s *p, int K) {
    const int R = p->radius;
    const double nx = (double)p->nx, ny = (double)p->ny;
    const int TX = star2d_tile_x(K, R);
    const double ly = std::min<double>(p->ly, ny);
    const double nstrips = std::ceil(nx / TX), nsegs = std::ceil(ny / ly);
    const double rows = ly + 2.0 * K * R;  // streamed per wavefront
    // stage s starts 2sR rows into the stream: sum over s of (rows - 2sR)
    const double stage_rows = K * (ly + (K - 1.0) * R);
    const double waves = nstrips * nsegs;
    // lane shifts: 2R per row, fused into the FMAs for R <= 4 (interior form)
    const double per_stage_row = kVec2D * (4.0 * R + 1.0) + (R <= 4 ? 0.0 : 2.0 * R) + kRowStage2D;
    const double per_wave = rows * kRow2D + stage_rows * per_stage_row;
    Pass s;
    s.t_valu = simd_time(waves, per_wave, waves_per_simd_2d(R, K));
    s.t_plane = 0.0;
    s.scale = 1.0 + kLyPenalty * std::max(0.0, ly / 64.0 - 1.0) * K / 8.0;
    // wind-up rows are re-read from HBM; the overlapped halo columns of
    // neighbouring strips mostly come from L2
    const double cells = nx * ny;
    s.t_hbm = (cells * 4.0 * (rows / ly) + cells * 4.0) / kHbmEff2D;
    return s;
}

Pass model_3d(const stencil_plan_s *p, int K) {
    const int R = p->radius;
    const double nx = (double)p->nx, ny = (double)p->ny, nz = (double)p->nz;
    const int vec = (K == p->K) ? p->vec : 4;
    const int wl = p->s3_lanes, nw = p->s3_rows;
    const double W = (double)wl * vec;
    const double nt = (double)nw * (64 / wl);
    const double ty = nt - 2.0 * K * R;
    double tx = nx, ntx = 1.0;
    if (nx > W || wl != 64) {
        const double hx = std::ceil((double)K * R / vec) * vec;
        tx = W - 2.0 * hx;
        ntx = std::ceil(nx / tx);
    }
    const double lz = std::min<double>(p->s3_lz, nz);
    const double nty = std::ceil(ny / ty), nseg = std::ceil(nz / lz);
    const double blocks = ntx * nty * nseg;
    const double planes = lz + 2.0 * K * R;
    // stage s starts 2sR planes into the stream
    const double stage_planes = K * (lz + (K - 1.0) * R);
    // load-only wavefronts: those whose rows all lie in the outer R rows
    const double rpw = 64.0 / wl;
    const double load_only = 2.0 * std::floor(R / rpw);
    const double compute = nw - load_only;
    const double per_stage_plane = vec * (6.0 * R + 1.0) + 2.0 * R + kRowStage3D;
    const double instr_block = planes * (compute * kRow3D + load_only * kLoadOnly3D) +
                               stage_planes * compute * per_stage_plane;
    double spill = 1.0;
    if (R >= 5 && K * R > 4) spill += kSpill * (K * R - 4.0) * (K * R - 4.0);
    if (R >= 4 && K > 1) spill += kSpillK * (K - 1.0) * R;
    Pass s;
    s.t_valu = blocks * instr_block * spill * kCyclesPerWaveInstr / (kCUs * kSimdPerCU * kClock);
    // one workgroup per CU at a time (1024 threads, <= 128 VGPRs): the
    // plane loop of each CU's blocks runs back to back, each plane its
    // SIMD's share of the issue plus the barrier/LDS latency
    const double waves_per_simd = std::ceil(nw / kSimdPerCU);
    const double issue_cycles = waves_per_simd * (instr_block / nw) * spill * kCyclesPerWaveInstr;
    const double rounds = std::ceil(blocks / kCUs);
    // one barrier and LDS round trip per plane, per pair of planes when paired
    const double barriers = p->s3_pair ? std::ceil(planes / 2.0) : planes;
    s.t_plane = rounds * (issue_cycles + barriers * kPlaneLatency3D) / kClock;
    const double cells = nx * ny * nz;
    s.t_hbm = (cells * 4.0 * (planes / lz) * (nt / ty) + cells * 4.0) / kHbmEff3D;
    return s;
}

// LDS-free single-step layout: no redundant cells, every wavefront
// independent; bounded by HBM (one read and one write per cell, plus the
// 2R wind-up planes of each segment) or by VALU issue (4 cells per lane:
// one FMA per point, 2R lane shifts, a per-row overhead).
constexpr double kRow3R = 12.0;

Pass model_3r(const stencil_plan_s *p) {
    const int R = p->radius;
    const double nx = (double)p->nx, ny = (double)p->ny, nz = (double)p->nz;
    const double lz = std::min<double>(p->s3_lz, nz);
    // a wavefront holds 64 / lpr row groups of lpr lanes (4 cells each)
    const double groups = 64.0 / p->s3_lpr;
    const double nstrips = std::ceil(nx / (4.0 * p->s3_lpr)), nyb = std::ceil(ny / (p->s3_rpl * groups));
    const double nseg = std::ceil(nz / lz);
    const double waves = nstrips * nyb * nseg;
    const double per_row = 4.0 * (6.0 * R + 1.0) + 2.0 * R + kRow3R;
    Pass s;
    s.t_valu = waves * lz * p->s3_rpl * per_row * kCyclesPerWaveInstr / (kCUs * kSimdPerCU * kClock);
    s.t_plane = 0.0;
    const double cells = nx * ny * nz;
    // the 2R neighbour rows of each centre plane come from L2 when the
    // neighbouring wavefronts loaded them moments before; the fraction that
    // misses grows with R (FETCH_SIZE on 512^3: 1.16x the algorithmic
    // reads at R = 1, 2.1-2.4x from R = 3 on with 2 or 4 rows per wavefront)
    const double miss = std::min(kMissMax, kMissSlope * (R - 1));
    const double reads = (lz + 2.0 * R) / lz * (1.0 + 2.0 * R * miss / p->s3_rpl);
    s.t_hbm = (cells * 4.0 * reads + cells * 4.0) / kHbmEff3D;
    return s;
}

}  // namespace

extern "C" int stencil_plan_model(stencil_plan_t plan, const char *config, double out[4]) {
    star_clear_error();
    if (!plan || !out) return star_set_error(STENCIL_EINVAL, "plan/out is NULL");
    stencil_plan_s trial = *plan;
    if (config && *config) {
        const int rc = plan_configure(&trial, config);
        if (rc != STENCIL_OK) return rc;
    }
    if (trial.variant == STAR_NAIVE || trial.storage != STENCIL_F32)
        return star_set_error(STENCIL_EUNSUPPORTED, "the model covers the FP32 streaming kernels");
    const Pass s = trial.ndim == 2 ? model_2d(&trial, trial.K)
                   : trial.s3_rpl > 0 ? model_3r(&trial)
                                      : model_3d(&trial, trial.K);
    const double t =
        (std::max({s.t_hbm, s.t_valu, s.t_plane}) + (trial.ndim == 2 ? kLaunch2D : kLaunch3D)) * s.scale;
    out[0] = (double)trial.ncells * trial.K / t / 1e9;
    out[1] = s.t_hbm * 1e6;
    out[2] = s.t_valu * 1e6;
    out[3] = s.t_plane * 1e6;
    return STENCIL_OK;
}
