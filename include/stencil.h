/*
 * stencil.h -- C ABI of the MI355X (gfx950) star-stencil library.
 *
 * The library applies repeated time steps of a 2D or 3D star stencil of
 * radius 1..8 (Zohouri, Podobas, Matsuoka, "High-Performance High-Order
 * Stencil Computation on FPGAs Using OpenCL", IPDPSW 2018, Sec. IV.A,
 * Eq. (1)):
 *
 *   f^{t+1}(p) = c_C f^t(p) + sum_{i=1..R} sum_{d} c_{d,i} f^t(clamp(p + i e_d))
 *
 * with d over W,E,S,N (2D) or W,E,S,N,B,A (3D): W/E = -x/+x, S/N = -y/+y,
 * B/A = -z/+z.  Out-of-grid neighbours take the value of the border cell
 * (Sec. III.B, Sec. IV.B), independently per axis, at every step.  The
 * kernels fuse several time steps per pass over memory (combined spatial and
 * temporal blocking with overlapped halos, Sec. III.A, Eq. (2)).
 *
 * Conventions shared by every entry point:
 *   - Grids are dense, row-major, x fastest: index = x + nx*(y + ny*z).
 *     dims[] is given in x, y[, z] order.
 *   - Coefficients are per point, in the order c_C, then for i = 1..R the
 *     directions W, E, S, N (, B, A): 1 + 2*ndim*R FP32 values.  They are
 *     copied at plan time; the caller keeps ownership of its array.
 *   - Grid pointers are DEVICE pointers owned by the caller.  The library
 *     never frees them and never writes the input grid.
 *   - Each FP32 cell update is evaluated as c_C*f_C followed by one fused
 *     multiply-add per neighbour in coefficient order, so every tuning of a
 *     plan gives the same bits.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Run calls only enqueue work and return; device faults surface on the
 *     caller's next synchronisation.
 *   - Every int-returning function returns STENCIL_OK (0) or a negative
 *     status; stencil_last_error() then describes the failure (per thread).
 *     No C++ exception crosses this interface.
 */
#ifndef MI355X_STENCIL_H
#define MI355X_STENCIL_H

#include <stddef.h>
#include <stdint.h>

#ifndef STENCIL_API
#define STENCIL_API __attribute__((visibility("default")))
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct stencil_plan_s *stencil_plan_t; /* opaque, library-owned */

enum stencil_status {
    STENCIL_OK = 0,
    STENCIL_EINVAL = -1,       /* bad argument (nothing was enqueued)        */
    STENCIL_ENOMEM = -2,       /* device or host allocation failed           */
    STENCIL_EDEVICE = -3,      /* a HIP call or kernel launch failed         */
    STENCIL_EUNSUPPORTED = -4, /* valid request the library does not support */
    STENCIL_EOVERFLOW = -5     /* a low-precision tile scale left its range  */
};

enum stencil_boundary {
    STENCIL_BOUNDARY_CLAMP = 0,  /* border cell replaces out-of-grid cells (Sec. III.B)     */
    STENCIL_BOUNDARY_PADDED = 1  /* fixed ghost frame of `radius` cells read from memory
                                    (the larger allocation of Sec. IV.B)                    */
};

enum stencil_storage {
    STENCIL_F32 = 0,         /* state kept in FP32 between passes                    */
    STENCIL_F16 = 1,         /* FP32 anchor + FP16 delta with per-tile 2^e scales    */
    STENCIL_BF16 = 2,        /* FP32 anchor + BF16 delta with per-tile 2^e scales    */
    STENCIL_F16_SCALED = 3,  /* state itself in FP16 with per-tile 2^e scales        */
    STENCIL_BF16_SCALED = 4  /* state itself in BF16 with per-tile 2^e scales        */
};

/*
 * Creates a plan for one grid shape, radius and coefficient set (Eq. (1)).
 *   plan     out: the new plan (set to NULL on failure).
 *   ndim     2 or 3.
 *   dims     ndim extents in x, y[, z] order, each >= 1; the cell count times
 *            4 bytes must fit in int64.
 *   radius   1..8.  The paper's diffusion stencils have radius 1..4; the
 *            higher radii follow its scaling discussion (Sec. VI.A).  In 3D
 *            at most 4/3/3/2/2/2/1/1 steps are fused per pass for radius
 *            1..8 (the row layout of single-step passes is the default at
 *            radius 6..8); low-precision storage is built for radius 1..4
 *            (EUNSUPPORTED above).
 *   coeffs   host array of ncoeffs FP32 values in the order given above.
 *   ncoeffs  must equal 1 + 2*ndim*radius.
 *   boundary STENCIL_BOUNDARY_CLAMP: every out-of-grid neighbour takes the
 *            nearest border cell (Sec. III.B).
 *            STENCIL_BOUNDARY_PADDED: the padded-halo arrangement of
 *            Sec. IV.B.  dims are the interior extents; every array the
 *            plan runs on holds (dims[a] + 2*radius) cells per axis, the
 *            interior at offset radius on every axis, inside a ghost frame
 *            of `radius` cells that is never updated: each step applies
 *            Eq. (1) to the interior cells with the neighbours read from the
 *            array (no clamp), and `out`'s frame is a copy of `in`'s.  FP32
 *            storage only (EUNSUPPORTED otherwise).
 * Allocates the plan's device scratch (one grid of FP32) on the current
 * device and picks a kernel configuration (from the tuning cache when one
 * is present, otherwise built-in defaults).  Errors: EINVAL, ENOMEM,
 * EDEVICE, EUNSUPPORTED.
 */
STENCIL_API int stencil_plan(stencil_plan_t *plan, int ndim, const int64_t *dims, int radius,
                 const float *coeffs, int ncoeffs, int boundary);

/*
 * A plan with shared coefficients (Sec. IV.A notes that the paper's
 * instance shares one coefficient per direction and optimises the case
 * where all differ; the comparison codes of Sec. VI.C share them): the two
 * neighbours at distance i along one axis share one coefficient.
 *   axis_coeffs  host array of 1 + ndim*radius FP32 values: c_C, then for
 *                i = 1..radius one value per axis, x, y (, z).
 *   ncoeffs      must equal 1 + ndim*radius.
 *   boundary     STENCIL_BOUNDARY_CLAMP (EUNSUPPORTED otherwise).
 *   radius       1..4 (EUNSUPPORTED above).
 * Each cell is evaluated in this fixed order, one rounding per operation:
 * c_C*f_C, then for i = 1..radius and each axis one fused multiply-add of
 * c_{a,i} with the rounded sum f(p - i e_a) + f(p + i e_a).  Exactly, this
 * is Eq. (1) with c_W,i = c_E,i = c_x,i and so on; the instruction count
 * per cell equals the per-point form's (one add replaces one FMA).  2D
 * plans fuse up to 4 steps per pass; 3D plans run the single-step row
 * layout.  FP32 storage.  Errors as stencil_plan.
 */
STENCIL_API int stencil_plan_symmetric(stencil_plan_t *plan, int ndim, const int64_t *dims,
                                       int radius, const float *axis_coeffs, int ncoeffs,
                                       int boundary, const char *tune);

/*
 * Expands the paper's per-direction coefficients (Sec. IV.A: one value per
 * direction, the same for every distance) into the per-point order of
 * stencil_plan: per_direction holds 1 + 2*ndim values c_C, c_W, c_E, c_S,
 * c_N (, c_B, c_A); out receives 1 + 2*ndim*radius values.  Host only.
 * Errors: EINVAL.
 */
STENCIL_API int stencil_coeffs_per_direction(int ndim, int radius, const float *per_direction,
                                             float *out);

/*
 * As stencil_plan, with extra controls:
 *   storage  STENCIL_F32, or one of the two low-precision forms (3D grids
 *            with nx % 4 == 0; not in the paper, which computes in FP32 only,
 *            Sec. IV.C).  Both store 16-bit codes q with one power-of-two
 *            scale per 64^3 tile (value = q * 2^e, e = ceil(log2 B) - 14 for
 *            a bound B on the tile's magnitude), compute every step in FP32
 *            and return FP32.
 *            STENCIL_F16 / STENCIL_BF16, anchored delta: an FP32 anchor A is
 *            fixed per window of anchor_m steps and only the delta D = F - A
 *            is stored; since one step S is linear, D evolves as
 *            D <- S D + G with G = S A - A computed once per window in FP32;
 *            A <- A + D at the window's end.
 *            STENCIL_F16_SCALED / STENCIL_BF16_SCALED, scaled state: the state
 *            itself is stored as codes between FP32 anchor steps (one FP32
 *            step every anchor_m steps re-derives the scales).
 *   anchor_m for the low-precision forms: steps per window (>= 1); ignored
 *            for F32.
 *   tune     NULL for automatic selection, or a configuration string of
 *            comma-separated items: "naive" (one thread per cell, one step
 *            per launch); 2D "k=" (fused steps, K*R <= 16, at most 10) and
 *            "ly=" (rows per segment); 3D "k=" (at most 4 for R = 1, 3 for
 *            R = 2, 3, 2 for R = 4..6, 1 for R = 7, 8),
 *            "wl=" (lanes per tile row, 32 or 64), "vec=" (cells per lane,
 *            4, or 8 for wl=64, k=1, R <= 2, aligned rows), "nw=" (waves per
 *            workgroup, <= 16), "lz=" (planes per segment) and "pair=1" (two
 *            planes per barrier, k=1, vec=4) for the xy-tile kernel; or the
 *            LDS-free single-step row layout: "rows=" (grid rows per
 *            wavefront: 1; 2; 4 for R <= 4), "nbp=" (0/1: neighbour rows
 *            loaded one plane ahead, R <= 4 with rows=1, 2), "lpr=" (lanes
 *            per grid row: 64, the default, or 16 -- four rows of a
 *            64-column strip per wavefront, for narrow grids; rows=1,
 *            nbp=0, R <= 4, per-point coefficients) and "lz=".  rows=2, 4
 *            and nbp=1 need nx % 4 == 0.  E.g. "k=4,ly=256" (2D),
 *            "k=2,wl=32,nw=16,lz=64", "k=1,rows=1,nbp=1,lz=128",
 *            "k=1,rows=1,nbp=0,lz=32,lpr=16" (3D).  Unknown keys or
 *            infeasible values give EINVAL.
 */
STENCIL_API int stencil_plan_ex(stencil_plan_t *plan, int ndim, const int64_t *dims, int radius,
                    const float *coeffs, int ncoeffs, int boundary, int storage,
                    int anchor_m, const char *tune);

/*
 * Applies `steps` time steps to the grid at `in` and writes f^steps to `out`.
 *   in, out  device pointers to nx*ny[*nz] floats (the padded extents for
 *            STENCIL_BOUNDARY_PADDED), 4-byte aligned; the two ranges must
 *            not overlap (EINVAL).  `in` is never written.
 *   steps    >= 0; 0 copies in to out.
 * Enqueues ceil(steps/K) passes on `stream`, ping-ponging between `out` and
 * the plan's scratch so that the last pass writes `out`.  A plan must not be
 * run concurrently with itself (its scratch is shared); distinct plans are
 * independent.  Errors: EINVAL, EDEVICE.
 */
STENCIL_API int stencil_run(stencil_plan_t plan, const float *in, float *out, int64_t steps, void *stream);

/* Largest grid, in cells, that stencil_run_noalloc accepts: 2^24 cells (a
 * 64 MiB FP32 partner grid, held on every device the call runs on until the
 * process ends). */
#define STENCIL_NOALLOC_MAX_CELLS 16777216

/*
 * stencil_run for callers that cannot allocate device memory while they run
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels, pass schedule and result, bit for bit, but
 * the ping-pong partner grid is a fixed device array of the library instead
 * of the plan's scratch, so the call performs no hipMalloc, hipFree or other
 * allocation.
 *   plan     an FP32-storage plan (EUNSUPPORTED otherwise) of at most
 *            STENCIL_NOALLOC_MAX_CELLS cells (EUNSUPPORTED otherwise).
 *   in, out  as for stencil_run; they must not overlap the static array.
 * The array's device address is looked up on the first call on each
 * device.  All calls on one device share that device's array: calls that
 * overlap in time on one device race, so order them (one stream, or
 * events).  Errors: EINVAL, EUNSUPPORTED, EDEVICE.
 */
STENCIL_API int stencil_run_noalloc(stencil_plan_t plan, const float *in, float *out, int64_t steps,
                                    void *stream);

/*
 * Runs n independent grids, grid g with plans[g], ins[g], outs[g] and
 * steps[g] (host arrays of length n, device grid pointers), with the same
 * result as n calls of stencil_run: every output is bitwise equal to its
 * own stencil_run.  The call builds a batch (see stencil_batch_create, with
 * default configuration) and launches it on `stream`; the batches of the
 * last 4 distinct calls are kept, so a repeated call (same plans, pointers
 * and steps) only replays its captured graph.  The grids run concurrently,
 * so no grid may write memory another grid reads or writes (EINVAL), and a
 * plan may appear only once.  n == 0 does nothing.  Errors: EINVAL, ENOMEM,
 * EDEVICE, EUNSUPPORTED.
 */
STENCIL_API int stencil_run_batched(int n, const stencil_plan_t *plans, const float *const *ins,
                        float *const *outs, const int64_t *steps, void *stream);

/*
 * The batched form as a reusable object.  Not in the paper, which runs one
 * grid at a time; this is the many-grids form of the same method: grids are
 * grouped into classes (dimension, radius, size: 2D grids of >= 2^18 cells
 * and 3D grids of >= 2^20 cells are "large"); each class has
 * one kernel configuration and runs as a chain of pass rounds (K fused steps
 * per round, a grid's last pass taking the remainder), each round one
 * launch of a persistent work-list kernel whose workgroups take
 * (grid, tile, segment) items from an atomic counter.  Class chains run
 * concurrently on side streams.  The whole schedule is captured into one
 * HIP graph at creation.
 *
 * stencil_batch_create: validates the grids as stencil_run_batched does and
 * builds the batch; the pointers and steps are fixed for its lifetime.
 *   tune  NULL, or a comma list of overrides: "2d.k=", "2d.ly=" (2D
 *         classes), "3d.k=", "3d.wl=" (32|64), "3d.vec=" (4|8), "3d.nw=",
 *         "3d.lz=" (3D classes) -- k is capped at the class's largest built
 *         K, vec=8 applies only to aligned single-step R <= 2 classes with
 *         wl=64 -- "streams=" (side streams, 1..16, default 4) and "graph="
 *         (1 = replay the captured graph, the default; 0 = enqueue the
 *         launches on every call) and "merge=0" (row-aligned grids keep
 *         classes of their own; by default they join the unaligned class
 *         of their kind: fewer, fuller pass rounds).  Without overrides a class takes its
 *         configuration from the tuning cache, else built-in defaults.
 *   Grids with steps == 0, low-precision storage, or 3D planes of 2^31
 *   bytes or more are run by their own plan inside the batch.
 *   Errors: EINVAL, ENOMEM, EDEVICE, EUNSUPPORTED.
 * stencil_batch_launch: enqueues one run of every grid on `stream`.  A batch
 *   must not run concurrently with itself (its counters and the plans'
 *   scratch are shared).  Errors: EINVAL, EDEVICE.
 * stencil_batch_autotune: times every feasible configuration of each class
 *   on the batch's own grids (class chains run alone on `stream`), keeps
 *   the fastest, records it in the tuning cache (STENCIL_TUNE_CACHE) and
 *   re-captures the graph.  The outputs hold the batch's result afterwards.
 *   report (NULL allowed): "<class> <config> <GCell/s>" lines.  Synchronises
 *   the device.  Errors: EINVAL, EDEVICE.
 * stencil_batch_describe: text summary (classes, configurations, rounds) into
 *   buf (NULL allowed); returns the full length.
 * stencil_batch_destroy: synchronises the device and frees the batch (not
 *   its plans or grids).  NULL is ignored.
 */
typedef struct stencil_batch_s *stencil_batch_t; /* opaque, library-owned */
STENCIL_API int stencil_batch_create(stencil_batch_t *batch, int n, const stencil_plan_t *plans,
                         const float *const *ins, float *const *outs, const int64_t *steps,
                         const char *tune);
STENCIL_API int stencil_batch_launch(stencil_batch_t batch, void *stream);
STENCIL_API int stencil_batch_autotune(stencil_batch_t batch, char *report, size_t report_len,
                           void *stream);
STENCIL_API int stencil_batch_describe(stencil_batch_t batch, char *buf, size_t len);
STENCIL_API void stencil_batch_destroy(stencil_batch_t batch);

/*
 * Analytic throughput model of the plan's kernel (the GPU counterpart of the
 * paper's performance model, Sec. V.A): a pass of K fused steps is bounded by
 * the largest of its HBM time (bytes / effective bandwidth), its VALU issue
 * time and (3D) its per-plane critical path, plus a launch cost.
 *   config  NULL for the plan's own configuration, or a configuration string
 *           as for stencil_plan_ex's tune (validated the same way).
 *   out     out[0] predicted GCell/s, out[1] HBM time per pass (us),
 *           out[2] VALU time per pass (us), out[3] time of the sequential
 *           path per pass (us: 3D planes streamed per CU; 2D rows streamed
 *           per wavefront when wavefronts are fewer than SIMDs).
 * Host-only (no device call).  Errors: EINVAL, EUNSUPPORTED (the naive
 * variant and the low-precision forms are not modelled).
 */
STENCIL_API int stencil_plan_model(stencil_plan_t plan, const char *config, double out[4]);

/*
 * Measured autotuning (the empirical counterpart of the paper's model-guided
 * parameter search, Sec. V.A): times every feasible configuration of the
 * plan -- temporal degree K, segment length, lanes and cells per row -- on
 * the caller's grids at the plan's real shape, with HIP events on `stream`,
 * keeps the fastest in the plan and, when the environment variable
 * STENCIL_TUNE_CACHE names a writable file, records it there; later plans
 * of the same problem (ndim, radius, storage, dims) read it back, and plans
 * of the same size class (ceil(log2 side) per axis) fall back to it.  When
 * STENCIL_TUNE_TOP=N (N >= 1) is set, only the N candidates the analytic
 * model (stencil_plan_model) ranks highest are timed.
 *   in, out  device grids as for stencil_run (`out` is overwritten).
 *   report   optional host buffer (NULL allowed) for a text table of the
 *            candidates: "<config> <GCell/s>" per line, best first.
 * Synchronises `stream`.  Errors: EINVAL, EDEVICE.
 */
STENCIL_API int stencil_plan_autotune(stencil_plan_t plan, const float *in, float *out,
                                      char *report, size_t report_len, void *stream);

/*
 * Reports the plan's configuration.  Any output pointer may be NULL.
 *   K          time steps fused per pass.
 *   tile       output tile extent in x, y, z (cells; z = 1 in 2D).
 *   vec        cells per lane along x.
 *   bytes_per_cell_step  algorithmic HBM bytes per cell update (8/K for F32).
 */
STENCIL_API int stencil_plan_query(stencil_plan_t plan, int *K, int tile[3], int *vec,
                       double *bytes_per_cell_step);

/*
 * Writes a human-readable description of the plan's configuration
 * ("variant=s2d R=1 K=4 ...") into buf (always NUL-terminated when
 * len > 0).  Returns the length it needed, or a negative status.
 */
STENCIL_API int stencil_plan_describe(stencil_plan_t plan, char *buf, size_t len);

/*
 * FP64 reductions on the device: out[0] = max|x - ref|, out[1] = max|ref|,
 * out[2] = sum of x (all accumulated in FP64).
 *   x    device array of n floats; ref device array of n doubles (may be
 *        NULL, then out[0] = out[1] = 0).
 *   out  HOST array of 3 doubles; the call synchronises `stream`.
 * A NaN in x or ref, or an infinity in x where ref is finite, makes out[0]
 * NaN or infinite (never silently skipped); a NaN in ref also makes out[1]
 * NaN; the sum carries NaN and infinities as FP64 addition does.
 * Errors: EINVAL, ENOMEM, EDEVICE.
 */
STENCIL_API int stencil_reduce_f64(const float *x, const double *ref, int64_t n, double out[3], void *stream);

/*
 * Releases the plan and its device scratch.  NULL is a no-op.  Waits for all
 * work on the plan's device first: runs are enqueued on caller streams the
 * plan does not record, and its scratch (and precision-form buffers) may be
 * in use on any of them; freeing device memory (hipFree) would wait for the
 * device anyway.  Destroy plans outside latency-critical loops.
 */
STENCIL_API void stencil_plan_destroy(stencil_plan_t plan);

/* Static text for a status code. */
STENCIL_API const char *stencil_status_string(int status);

/* Text of the last failure on the calling thread ("" when none). */
STENCIL_API const char *stencil_last_error(void);

/* Library version string. */
STENCIL_API const char *stencil_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MI355X_STENCIL_H */
