// plan.hpp -- the plan object behind stencil_plan_t (internal).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "common.hpp"

enum star_variant : int {
    STAR_NAIVE = 0,  // one thread per cell, one step per launch
    STAR_S2D = 1,    // 2D x-strip / y-stream, K fused steps
    STAR_S3D = 2,    // 3D xy-tile in LDS / z-stream, K fused steps
};

struct LowpState;  // precision-form buffers (lowp.cpp)

struct stencil_plan_s {
    // problem
    int ndim = 2;
    int64_t nx = 1, ny = 1, nz = 1, ncells = 1;
    int radius = 1;
    int npts = 5;
    star::Coefs cf{};
    int storage = 0;
    int anchor_m = 0;
    int pad = 0;               // padded-halo boundary: frame width (= R); nx, ny, nz include it
    int sym = 0;               // shared coefficients per axis and distance (cf: 1 + ndim*R values)
    int device = 0;
    uint64_t serial = 0;       // unique per plan created in this process
    float *scratch = nullptr;  // one FP32 grid, ping-pong partner of `out` (the anchor for F16/BF16)
    LowpState *lowp = nullptr; // low-precision state when storage != F32

    // configuration
    int variant = STAR_NAIVE;
    int K = 1;        // steps fused per pass
    int ly = 0;       // 2D: output rows per y-segment
    int tile[3] = {1, 1, 1};
    int vec = 1;
    // 3D streaming kernel
    int s3_lanes = 32;  // lanes along x per tile row
    int s3_rows = 16;   // tile rows (halo included) per workgroup
    int s3_lz = 64;     // output planes per z-segment
    int s3_pair = 0;    // 1: two planes per barrier (single-step passes)
    int s3_rpl = 0;     // > 0: LDS-free single-step layout, grid rows per wavefront
    int s3_nbp = 0;     // rows layout: neighbour rows loaded one plane ahead
    int s3_lpr = 64;    // rows layout: lanes per grid row (64, or 16 for narrow grids)
    std::string tuned_by = "default";
};

// Chooses the kernel configuration; `tune` may override it (NULL = auto).
int plan_configure(stencil_plan_s *p, const char *tune);
// Enqueues `steps` time steps from in to out (passes ping-pong between out
// and the plan's scratch; the last pass writes out).
hipError_t plan_enqueue(const stencil_plan_s *p, const float *in, float *out, int64_t steps,
                        hipStream_t stream);
// Configuration recorded for this problem in the tuning cache, if any.
bool tune_cache_lookup(const stencil_plan_s *p, std::string &config);
// The tuning cache (file named by STENCIL_TUNE_CACHE): lines of
// "<key>\t<config>\t<GCell/s>"; the last line of a key wins.
bool tune_cache_get(const std::string &key, std::string &config);
void tune_cache_put(const std::string &key, const std::string &config, double gcells);
// Base architecture name of a device ("gfx950"), "unknown" if unavailable.
std::string tune_arch_name(int device);
// Splits `steps` into the K of each pass.
void plan_pass_schedule(const stencil_plan_s *p, int64_t steps, std::vector<int> &passes);
// Enqueues one pass of `k` fused steps from src to dst.
hipError_t plan_launch_pass(const stencil_plan_s *p, int k, const float *src, float *dst,
                            hipStream_t stream);
std::string plan_describe(const stencil_plan_s *p);
std::string plan_describe_config(const stencil_plan_s *p);
void plan_release_extra(stencil_plan_s *p);

// Precision form (lowp.cpp): device state, and the run schedule.
int lowp_allocate(stencil_plan_s *p);
void lowp_release(stencil_plan_s *p);
hipError_t lowp_enqueue(const stencil_plan_s *p, const float *in, float *out, int64_t steps,
                        hipStream_t stream);

// Checks the arguments of one stencil_run (also used per grid of a batch).
int run_check(const stencil_plan_s *plan, const float *in, float *out, int64_t steps);

// Records a failure for stencil_last_error() and returns status.
int star_set_error(int status, const char *msg);
void star_clear_error();
