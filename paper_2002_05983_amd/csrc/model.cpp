// model.cpp -- analytic throughput model of the streaming kernels.
//
// The paper sizes its FPGA design with a performance model before building
// the top candidates (Sec. V.A).  This is the GPU counterpart for the kernels
// here: a pass of K fused steps is bounded by the largest of
//   HBM     bytes the pass must move / effective bandwidth;
//   VALU    wavefront instructions / (CUs x SIMDs), 4 cycles per wave64
//           instruction on a 16-lane SIMD;
//   stream  the sequential path: (3D) the per-plane critical path of a
//           workgroup -- its VALU issue, LDS write, barrier, LDS reads --
//           times the planes each CU streams one after the other; (2D) the
//           rows a wavefront streams alone when there are fewer wavefronts
//           than SIMDs;
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
// Fitted to the autotuner's measurements on MI355X (every candidate of 13
// problems: 2D 16384^2 and 4096^2, 3D 512^3, 768^3 and 192x256x320) by a
// grid search minimising mean |log(predicted / measured)|:
constexpr double kHbmEff2D = 5.0e12, kHbmEff3D = 5.0e12;  // B/s reached by the passes
// s per pass: launch, plus (2D) the ramp-up and drain of the last wavefronts
constexpr double kLaunch2D = 30e-6, kLaunch3D = 2e-6;
// instructions per wavefront row and stage beyond the FMAs and lane shifts
// (clamps, register moves, index arithmetic), and per streamed row
constexpr double kRowStage2D = 10.0, kRow2D = 16.0;
constexpr double kRowStage3D = 25.0, kRow3D = 24.0, kLoadOnly3D = 20.0;
// per-plane critical path of a 3D workgroup beyond its VALU issue time
// (LDS write, barrier, LDS reads), cycles
constexpr double kPlaneLatency3D = 400.0;

struct Pass {
    double t_hbm, t_valu, t_plane;
};

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
    const double instr = waves * per_wave;
    Pass s;
    s.t_valu = instr * kCyclesPerWaveInstr / (kCUs * kSimdPerCU * kClock);
    // few wavefronts: each streams its rows alone on its SIMD
    s.t_plane = std::ceil(waves / (kCUs * kSimdPerCU)) * per_wave * kCyclesPerWaveInstr / kClock;
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
    Pass s;
    s.t_valu = blocks * instr_block * kCyclesPerWaveInstr / (kCUs * kSimdPerCU * kClock);
    // one workgroup per CU at a time (1024 threads, <= 128 VGPRs): the
    // plane loop of each CU's blocks runs back to back, each plane its
    // SIMD's share of the issue plus the barrier/LDS latency
    const double waves_per_simd = std::ceil(nw / kSimdPerCU);
    const double issue_cycles = waves_per_simd * (instr_block / nw) * kCyclesPerWaveInstr;
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
    const double nstrips = std::ceil(nx / 256.0), nyb = std::ceil(ny / p->s3_rpl);
    const double nseg = std::ceil(nz / lz);
    const double waves = nstrips * nyb * nseg;
    const double per_row = 4.0 * (6.0 * R + 1.0) + 2.0 * R + kRow3R;
    Pass s;
    s.t_valu = waves * lz * p->s3_rpl * per_row * kCyclesPerWaveInstr / (kCUs * kSimdPerCU * kClock);
    s.t_plane = 0.0;
    const double cells = nx * ny * nz;
    // the 2R neighbour rows of each centre plane come from L2 when the
    // neighbouring wavefronts loaded them moments before; the fraction that
    // misses grows with R (FETCH_SIZE on 512^3: 2.2-3.1x the algorithmic
    // reads at R = 3, 4; near 1x at R = 1)
    const double miss = std::min(0.3, 0.1 * (R - 1));
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
        std::max({s.t_hbm, s.t_valu, s.t_plane}) + (trial.ndim == 2 ? kLaunch2D : kLaunch3D);
    out[0] = (double)trial.ncells * trial.K / t / 1e9;
    out[1] = s.t_hbm * 1e6;
    out[2] = s.t_valu * 1e6;
    out[3] = s.t_plane * 1e6;
    return STENCIL_OK;
}
