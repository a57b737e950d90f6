/*
 * star_oracle.c -- plain CPU reference for repeated star-stencil sweeps.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path links,
 * loads or calls this file; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark do.  It shares no code, header or table
 * with the GPU library.
 *
 * What it computes -- Zohouri, Podobas, Matsuoka, "High-Performance
 * High-Order Stencil Computation on FPGAs Using OpenCL" (IPDPSW 2018):
 *
 *   Sec. IV.A, Eq. (1): one time step of a star stencil of radius `rad`
 *     f^{t+1}(p) = c_C f^t(p)
 *                + sum_{i=1..rad} sum_{d in W,E,S,N[,B,A]} c_{d,i} f^t(p + i*e_d)
 *   The 2D form drops the Below/Above neighbours (Sec. IV.A).  The printed
 *   sum starts at i = 0; it is read as i = 1..rad, because the paper counts
 *   12*rad+1 FLOP (6*rad+1 multiplies, 6*rad adds) per 3D update, which
 *   leaves no room for an i = 0 term.
 *   Coefficients are taken per point (Sec. IV.A: all coefficients treated as
 *   different), in the order: c_C, then for i = 1..rad the directions
 *   W, E, S, N (, B, A).  W/E are -x/+x, S/N are -y/+y, B/A are -z/+z, with
 *   x the contiguous axis.
 *
 *   Sec. III.B and IV.B: an out-of-grid neighbour takes the value of the
 *   cell on the border, i.e. each coordinate is clamped to [0, n-1]
 *   independently, at every step, against the current field.
 *
 * Entry points:
 *   oracle_star_run_f64  -- the definition in double precision: the oracle.
 *   oracle_star_run_f32  -- the same definition evaluated in single
 *     precision with one fixed operation order (the centre product first,
 *     then one fused multiply-add per neighbour in the coefficient order
 *     above).  Used to check that a single-precision implementation that
 *     keeps this order reproduces it bit for bit.
 *   oracle_star_sample_f64 / _f32 -- the same values at chosen cells, each
 *     from its own dependence cone.
 *   oracle_star_run_padded_f64 / _f32 -- the padded-halo boundary of
 *     Sec. IV.B (fixed ghost frame of width rad, read without clamping).
 *   oracle_star_run_sym_f32 -- shared coefficients per axis and distance,
 *     single precision, with the pair sum f_- + f_+ rounded first.
 *
 * Layout: dense, row-major, x fastest: index = x + nx*(y + ny*z).  For 2D,
 * dims[2] is ignored (nz = 1).
 *
 * Build: cc -O3 -fopenmp -ffp-contract=off -shared -fPIC (contraction off so
 * the single-precision form keeps exactly the operations written here).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline int64_t clamp_index(int64_t v, int64_t n)
{
    if (v < 0) return 0;
    if (v >= n) return n - 1;
    return v;
}

static int check_args(int ndim, const int64_t *dims, int rad, int ncoef,
                      int64_t steps, int64_t *nx, int64_t *ny, int64_t *nz)
{
    if (ndim != 2 && ndim != 3) return -1;
    if (rad < 1 || rad > 64) return -1;
    if (ncoef != 1 + 2 * ndim * rad) return -1;
    if (steps < 0) return -1;
    *nx = dims[0];
    *ny = dims[1];
    *nz = (ndim == 3) ? dims[2] : 1;
    if (*nx < 1 || *ny < 1 || *nz < 1) return -1;
    return 0;
}

/*
 * One step of Eq. (1) with the clamp boundary, in double precision.
 *
 * The sum is evaluated one grid row at a time: every cell of the row starts
 * from the centre product c_C*f(p), then each neighbour term is added in the
 * coefficient order (for i = 1..rad: W, E, S, N[, B, A]).  Each cell thus
 * sees exactly the operations and order of the per-cell sum; only the loop
 * over the cells of a row is moved inside the loop over terms, so that the
 * compiler can vectorise it.  The x-neighbours are read from a copy of the
 * row with `rad` border values repeated at each end (the clamp along x); the
 * y- and z-neighbours are whole rows whose row index is clamped.
 */
static int step_f64(int ndim, int64_t nx, int64_t ny, int64_t nz, int rad,
                     const double *c, const double *src, double *dst, int nthreads)
{
    int status = 0;
#pragma omp parallel num_threads(nthreads)
    {
        double *padded = (double *)malloc((size_t)(nx + 2 * rad) * sizeof(double));
        if (!padded) {
#pragma omp atomic write
            status = -2;
        }
#pragma omp for collapse(2) schedule(static)
        for (int64_t z = 0; z < nz; ++z) {
            for (int64_t y = 0; y < ny; ++y) {
                if (!padded) continue;
#define ROW(yy, zz) (src + nx * ((yy) + ny * (zz)))
                const double *row = ROW(y, z);
                double *out = dst + nx * (y + ny * z);
                for (int64_t x = -rad; x < nx + rad; ++x)
                    padded[x + rad] = row[clamp_index(x, nx)];
                const double *f = padded + rad;   /* f[x - i] .. f[x + i] valid */
                for (int64_t x = 0; x < nx; ++x) out[x] = c[0] * f[x];
                int k = 1;
                for (int i = 1; i <= rad; ++i) {
                    const double cw = c[k++], ce = c[k++], cs = c[k++], cn = c[k++];
                    const double *south = ROW(clamp_index(y - i, ny), z);
                    const double *north = ROW(clamp_index(y + i, ny), z);
                    for (int64_t x = 0; x < nx; ++x) out[x] += cw * f[x - i];      /* W */
                    for (int64_t x = 0; x < nx; ++x) out[x] += ce * f[x + i];      /* E */
                    for (int64_t x = 0; x < nx; ++x) out[x] += cs * south[x];     /* S */
                    for (int64_t x = 0; x < nx; ++x) out[x] += cn * north[x];     /* N */
                    if (ndim == 3) {
                        const double cb = c[k++], ca = c[k++];
                        const double *below = ROW(y, clamp_index(z - i, nz));
                        const double *above = ROW(y, clamp_index(z + i, nz));
                        for (int64_t x = 0; x < nx; ++x) out[x] += cb * below[x];  /* B */
                        for (int64_t x = 0; x < nx; ++x) out[x] += ca * above[x];  /* A */
                    }
                }
#undef ROW
            }
        }
        free(padded);
    }
    return status;
}

/* The same step in single precision: the centre product, then one fmaf per
 * neighbour in coefficient order (same row-at-a-time evaluation). */
static int step_f32(int ndim, int64_t nx, int64_t ny, int64_t nz, int rad,
                    const float *c, const float *src, float *dst, int nthreads)
{
    int status = 0;
#pragma omp parallel num_threads(nthreads)
    {
        float *padded = (float *)malloc((size_t)(nx + 2 * rad) * sizeof(float));
        if (!padded) {
#pragma omp atomic write
            status = -2;
        }
#pragma omp for collapse(2) schedule(static)
        for (int64_t z = 0; z < nz; ++z) {
            for (int64_t y = 0; y < ny; ++y) {
                if (!padded) continue;
#define ROW(yy, zz) (src + nx * ((yy) + ny * (zz)))
                const float *row = ROW(y, z);
                float *out = dst + nx * (y + ny * z);
                for (int64_t x = -rad; x < nx + rad; ++x)
                    padded[x + rad] = row[clamp_index(x, nx)];
                const float *f = padded + rad;
                for (int64_t x = 0; x < nx; ++x) out[x] = c[0] * f[x];
                int k = 1;
                for (int i = 1; i <= rad; ++i) {
                    const float cw = c[k++], ce = c[k++], cs = c[k++], cn = c[k++];
                    const float *south = ROW(clamp_index(y - i, ny), z);
                    const float *north = ROW(clamp_index(y + i, ny), z);
                    for (int64_t x = 0; x < nx; ++x) out[x] = fmaf(cw, f[x - i], out[x]);
                    for (int64_t x = 0; x < nx; ++x) out[x] = fmaf(ce, f[x + i], out[x]);
                    for (int64_t x = 0; x < nx; ++x) out[x] = fmaf(cs, south[x], out[x]);
                    for (int64_t x = 0; x < nx; ++x) out[x] = fmaf(cn, north[x], out[x]);
                    if (ndim == 3) {
                        const float cb = c[k++], ca = c[k++];
                        const float *below = ROW(y, clamp_index(z - i, nz));
                        const float *above = ROW(y, clamp_index(z + i, nz));
                        for (int64_t x = 0; x < nx; ++x) out[x] = fmaf(cb, below[x], out[x]);
                        for (int64_t x = 0; x < nx; ++x) out[x] = fmaf(ca, above[x], out[x]);
                    }
                }
#undef ROW
            }
        }
        free(padded);
    }
    return status;
}

/*
 * Runs `steps` time steps from f0 and writes f^steps to out.
 * f0 and out are host arrays of nx*ny*nz doubles; they may alias.
 * Returns 0, or -1 on bad arguments, -2 when memory runs out.
 */
int oracle_star_run_f64(int ndim, const int64_t *dims, int rad,
                        const double *coef, int ncoef,
                        const double *f0, double *out, int64_t steps,
                        int nthreads)
{
    int64_t nx, ny, nz;
    if (check_args(ndim, dims, rad, ncoef, steps, &nx, &ny, &nz)) return -1;
    if (nthreads < 1) nthreads = 1;
    size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
    double *a = (double *)malloc(n * sizeof(double));
    double *b = (double *)malloc(n * sizeof(double));
    if (!a || !b) { free(a); free(b); return -2; }
    memcpy(a, f0, n * sizeof(double));
    for (int64_t t = 0; t < steps; ++t) {
        if (step_f64(ndim, nx, ny, nz, rad, coef, a, b, nthreads)) {
            free(a); free(b);
            return -2;
        }
        double *tmp = a; a = b; b = tmp;
    }
    memcpy(out, a, n * sizeof(double));
    free(a);
    free(b);
    return 0;
}

/* Single-precision counterpart of oracle_star_run_f64 (same contract). */
int oracle_star_run_f32(int ndim, const int64_t *dims, int rad,
                        const float *coef, int ncoef,
                        const float *f0, float *out, int64_t steps,
                        int nthreads)
{
    int64_t nx, ny, nz;
    if (check_args(ndim, dims, rad, ncoef, steps, &nx, &ny, &nz)) return -1;
    if (nthreads < 1) nthreads = 1;
    size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
    float *a = (float *)malloc(n * sizeof(float));
    float *b = (float *)malloc(n * sizeof(float));
    if (!a || !b) { free(a); free(b); return -2; }
    memcpy(a, f0, n * sizeof(float));
    for (int64_t t = 0; t < steps; ++t) {
        if (step_f32(ndim, nx, ny, nz, rad, coef, a, b, nthreads)) {
            free(a); free(b);
            return -2;
        }
        float *tmp = a; a = b; b = tmp;
    }
    memcpy(out, a, n * sizeof(float));
    free(a);
    free(b);
    return 0;
}

/*
 * Value of f^steps at a list of cells, computed from the dependence cone of
 * each cell only (the cells within steps*rad of it along every axis, with
 * the clamp applied at every step).  This lets a full-size run be checked at
 * sampled cells without sweeping the whole grid.  cells holds (x, y[, z])
 * triples (z ignored in 2D); results go to vals.  Returns 0, -1, or -2.
 */
int oracle_star_sample_f64(int ndim, const int64_t *dims, int rad,
                           const double *coef, int ncoef,
                           const float *f0, int64_t steps,
                           const int64_t *cells, int64_t ncells,
                           double *vals, int nthreads)
{
    int64_t nx, ny, nz;
    if (check_args(ndim, dims, rad, ncoef, steps, &nx, &ny, &nz)) return -1;
    if (nthreads < 1) nthreads = 1;
    int status = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t q = 0; q < ncells; ++q) {
        int64_t p[3] = {cells[3 * q], cells[3 * q + 1], ndim == 3 ? cells[3 * q + 2] : 0};
        int64_t n3[3] = {nx, ny, nz};
        /* Box [lo, hi) of the dependence cone, clipped to the grid: clipping
         * is exact because clamped reads never leave the grid. */
        int64_t lo[3], hi[3], ext[3];
        for (int a = 0; a < 3; ++a) {
            int64_t reach = (a < ndim) ? steps * (int64_t)rad : 0;
            lo[a] = p[a] - reach < 0 ? 0 : p[a] - reach;
            hi[a] = p[a] + reach + 1 > n3[a] ? n3[a] : p[a] + reach + 1;
            ext[a] = hi[a] - lo[a];
        }
        size_t m = (size_t)ext[0] * ext[1] * ext[2];
        double *a = (double *)malloc(m * sizeof(double));
        double *b = (double *)malloc(m * sizeof(double));
        if (!a || !b) {
            free(a); free(b);
#pragma omp atomic write
            status = -2;
            continue;
        }
        for (int64_t z = 0; z < ext[2]; ++z)
            for (int64_t y = 0; y < ext[1]; ++y)
                for (int64_t x = 0; x < ext[0]; ++x)
                    a[x + ext[0] * (y + ext[1] * z)] =
                        (double)f0[(lo[0] + x) + nx * ((lo[1] + y) + ny * (lo[2] + z))];
        /* At step t, only cells within (steps - t - 1)*rad of p matter; the
         * box shrinks accordingly, but cells near the clipped faces still
         * need their clamped neighbours, which stay inside the box because
         * the box reaches the grid border there. */
        for (int64_t t = 0; t < steps; ++t) {
            int64_t keep = (steps - t - 1) * (int64_t)rad;
            int64_t l2[3], h2[3];
            for (int ax = 0; ax < 3; ++ax) {
                int64_t r = (ax < ndim) ? keep : 0;
                l2[ax] = p[ax] - r < lo[ax] ? lo[ax] : p[ax] - r;
                h2[ax] = p[ax] + r + 1 > hi[ax] ? hi[ax] : p[ax] + r + 1;
            }
            for (int64_t z = l2[2]; z < h2[2]; ++z)
                for (int64_t y = l2[1]; y < h2[1]; ++y)
                    for (int64_t x = l2[0]; x < h2[0]; ++x) {
#define G(xx, yy, zz) a[((xx) - lo[0]) + ext[0] * (((yy) - lo[1]) + ext[1] * ((zz) - lo[2]))]
                        double acc = coef[0] * G(x, y, z);
                        int k = 1;
                        for (int i = 1; i <= rad; ++i) {
                            acc += coef[k++] * G(clamp_index(x - i, nx), y, z);
                            acc += coef[k++] * G(clamp_index(x + i, nx), y, z);
                            acc += coef[k++] * G(x, clamp_index(y - i, ny), z);
                            acc += coef[k++] * G(x, clamp_index(y + i, ny), z);
                            if (ndim == 3) {
                                acc += coef[k++] * G(x, y, clamp_index(z - i, nz));
                                acc += coef[k++] * G(x, y, clamp_index(z + i, nz));
                            }
                        }
                        b[(x - lo[0]) + ext[0] * ((y - lo[1]) + ext[1] * (z - lo[2]))] = acc;
#undef G
                    }
            double *tmp = a; a = b; b = tmp;
        }
        vals[q] = a[(p[0] - lo[0]) + ext[0] * ((p[1] - lo[1]) + ext[1] * (p[2] - lo[2]))];
        free(a);
        free(b);
    }
    return status;
}

/*
 * Single-precision counterpart of oracle_star_sample_f64: f^steps at the
 * given cells, each from its own dependence cone, with the operations and
 * order of oracle_star_run_f32 (so every sampled value equals the one the
 * full-grid single-precision run gives, bit for bit).
 */
int oracle_star_sample_f32(int ndim, const int64_t *dims, int rad,
                           const float *coef, int ncoef,
                           const float *f0, int64_t steps,
                           const int64_t *cells, int64_t ncells,
                           float *vals, int nthreads)
{
    int64_t nx, ny, nz;
    if (check_args(ndim, dims, rad, ncoef, steps, &nx, &ny, &nz)) return -1;
    if (nthreads < 1) nthreads = 1;
    int status = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t q = 0; q < ncells; ++q) {
        int64_t p[3] = {cells[3 * q], cells[3 * q + 1], ndim == 3 ? cells[3 * q + 2] : 0};
        int64_t n3[3] = {nx, ny, nz};
        int64_t lo[3], hi[3], ext[3];
        for (int a = 0; a < 3; ++a) {
            int64_t reach = (a < ndim) ? steps * (int64_t)rad : 0;
            lo[a] = p[a] - reach < 0 ? 0 : p[a] - reach;
            hi[a] = p[a] + reach + 1 > n3[a] ? n3[a] : p[a] + reach + 1;
            ext[a] = hi[a] - lo[a];
        }
        size_t m = (size_t)ext[0] * ext[1] * ext[2];
        float *a = (float *)malloc(m * sizeof(float));
        float *b = (float *)malloc(m * sizeof(float));
        if (!a || !b) {
            free(a); free(b);
#pragma omp atomic write
            status = -2;
            continue;
        }
        for (int64_t z = 0; z < ext[2]; ++z)
            for (int64_t y = 0; y < ext[1]; ++y)
                for (int64_t x = 0; x < ext[0]; ++x)
                    a[x + ext[0] * (y + ext[1] * z)] =
                        f0[(lo[0] + x) + nx * ((lo[1] + y) + ny * (lo[2] + z))];
        for (int64_t t = 0; t < steps; ++t) {
            int64_t keep = (steps - t - 1) * (int64_t)rad;
            int64_t l2[3], h2[3];
            for (int ax = 0; ax < 3; ++ax) {
                int64_t r = (ax < ndim) ? keep : 0;
                l2[ax] = p[ax] - r < lo[ax] ? lo[ax] : p[ax] - r;
                h2[ax] = p[ax] + r + 1 > hi[ax] ? hi[ax] : p[ax] + r + 1;
            }
            for (int64_t z = l2[2]; z < h2[2]; ++z)
                for (int64_t y = l2[1]; y < h2[1]; ++y)
                    for (int64_t x = l2[0]; x < h2[0]; ++x) {
#define G(xx, yy, zz) a[((xx) - lo[0]) + ext[0] * (((yy) - lo[1]) + ext[1] * ((zz) - lo[2]))]
                        float acc = coef[0] * G(x, y, z);
                        int k = 1;
                        for (int i = 1; i <= rad; ++i) {
                            acc = fmaf(coef[k], G(clamp_index(x - i, nx), y, z), acc); ++k;
                            acc = fmaf(coef[k], G(clamp_index(x + i, nx), y, z), acc); ++k;
                            acc = fmaf(coef[k], G(x, clamp_index(y - i, ny), z), acc); ++k;
                            acc = fmaf(coef[k], G(x, clamp_index(y + i, ny), z), acc); ++k;
                            if (ndim == 3) {
                                acc = fmaf(coef[k], G(x, y, clamp_index(z - i, nz)), acc); ++k;
                                acc = fmaf(coef[k], G(x, y, clamp_index(z + i, nz)), acc); ++k;
                            }
                        }
                        b[(x - lo[0]) + ext[0] * ((y - lo[1]) + ext[1] * (z - lo[2]))] = acc;
#undef G
                    }
            float *tmp = a; a = b; b = tmp;
        }
        vals[q] = a[(p[0] - lo[0]) + ext[0] * ((p[1] - lo[1]) + ext[1] * (p[2] - lo[2]))];
        free(a);
        free(b);
    }
    return status;
}

/*
 * Padded-halo boundary (the YASK arrangement of Sec. IV.B: a larger grid is
 * allocated and out-of-bound neighbours are read from memory rather than
 * clamped).  The arrays hold the interior of dims[] cells per axis inside a
 * frame of `rad` ghost cells on every side, so each axis has dims[a] + 2*rad
 * cells; index = x + px*(y + py*z) over the padded sizes px, py(, pz).  The
 * ghost frame holds fixed values (it is never updated): every step applies
 * Eq. (1) to the interior cells, reading neighbours straight from the padded
 * array with no clamp, and copies the frame unchanged.  Same arithmetic and
 * order as the clamp forms above (FP64; FP32 with the centre product, then
 * one fmaf per neighbour in coefficient order).
 */
static int padded_dims(int ndim, const int64_t *dims, int rad, int ncoef, int64_t steps,
                       int64_t *px, int64_t *py, int64_t *pz)
{
    int64_t nx, ny, nz;
    if (check_args(ndim, dims, rad, ncoef, steps, &nx, &ny, &nz)) return -1;
    *px = nx + 2 * (int64_t)rad;
    *py = ny + 2 * (int64_t)rad;
    *pz = (ndim == 3) ? nz + 2 * (int64_t)rad : 1;
    return 0;
}

static void step_padded_f64(int ndim, int64_t px, int64_t py, int64_t pz, int rad,
                            const double *c, const double *src, double *dst, int nthreads)
{
    const int64_t z0 = (ndim == 3) ? rad : 0, z1 = (ndim == 3) ? pz - rad : 1;
#pragma omp parallel for collapse(2) schedule(static) num_threads(nthreads)
    for (int64_t z = 0; z < pz; ++z) {
        for (int64_t y = 0; y < py; ++y) {
#define F(xx, yy, zz) src[(xx) + px * ((yy) + py * (zz))]
            for (int64_t x = 0; x < px; ++x) {
                const int inside = x >= rad && x < px - rad && y >= rad && y < py - rad &&
                                   z >= z0 && z < z1;
                if (!inside) {  /* ghost frame: fixed */
                    dst[x + px * (y + py * z)] = F(x, y, z);
                    continue;
                }
                double acc = c[0] * F(x, y, z);
                int k = 1;
                for (int i = 1; i <= rad; ++i) {
                    acc += c[k++] * F(x - i, y, z);   /* W */
                    acc += c[k++] * F(x + i, y, z);   /* E */
                    acc += c[k++] * F(x, y - i, z);   /* S */
                    acc += c[k++] * F(x, y + i, z);   /* N */
                    if (ndim == 3) {
                        acc += c[k++] * F(x, y, z - i); /* B */
                        acc += c[k++] * F(x, y, z + i); /* A */
                    }
                }
                dst[x + px * (y + py * z)] = acc;
            }
#undef F
        }
    }
}

static void step_padded_f32(int ndim, int64_t px, int64_t py, int64_t pz, int rad,
                            const float *c, const float *src, float *dst, int nthreads)
{
    const int64_t z0 = (ndim == 3) ? rad : 0, z1 = (ndim == 3) ? pz - rad : 1;
#pragma omp parallel for collapse(2) schedule(static) num_threads(nthreads)
    for (int64_t z = 0; z < pz; ++z) {
        for (int64_t y = 0; y < py; ++y) {
#define F(xx, yy, zz) src[(xx) + px * ((yy) + py * (zz))]
            for (int64_t x = 0; x < px; ++x) {
                const int inside = x >= rad && x < px - rad && y >= rad && y < py - rad &&
                                   z >= z0 && z < z1;
                if (!inside) {
                    dst[x + px * (y + py * z)] = F(x, y, z);
                    continue;
                }
                float acc = c[0] * F(x, y, z);
                int k = 1;
                for (int i = 1; i <= rad; ++i) {
                    acc = fmaf(c[k], F(x - i, y, z), acc); ++k;
                    acc = fmaf(c[k], F(x + i, y, z), acc); ++k;
                    acc = fmaf(c[k], F(x, y - i, z), acc); ++k;
                    acc = fmaf(c[k], F(x, y + i, z), acc); ++k;
                    if (ndim == 3) {
                        acc = fmaf(c[k], F(x, y, z - i), acc); ++k;
                        acc = fmaf(c[k], F(x, y, z + i), acc); ++k;
                    }
                }
                dst[x + px * (y + py * z)] = acc;
            }
#undef F
        }
    }
}

/* `steps` steps of the padded-halo form; f0 and out hold the padded arrays
 * (they may alias).  Returns 0, -1 on bad arguments, -2 when memory runs out. */
int oracle_star_run_padded_f64(int ndim, const int64_t *dims, int rad,
                               const double *coef, int ncoef,
                               const double *f0, double *out, int64_t steps,
                               int nthreads)
{
    int64_t px, py, pz;
    if (padded_dims(ndim, dims, rad, ncoef, steps, &px, &py, &pz)) return -1;
    if (nthreads < 1) nthreads = 1;
    size_t n = (size_t)px * (size_t)py * (size_t)pz;
    double *a = (double *)malloc(n * sizeof(double));
    double *b = (double *)malloc(n * sizeof(double));
    if (!a || !b) { free(a); free(b); return -2; }
    memcpy(a, f0, n * sizeof(double));
    for (int64_t t = 0; t < steps; ++t) {
        step_padded_f64(ndim, px, py, pz, rad, coef, a, b, nthreads);
        double *tmp = a; a = b; b = tmp;
    }
    memcpy(out, a, n * sizeof(double));
    free(a);
    free(b);
    return 0;
}

int oracle_star_run_padded_f32(int ndim, const int64_t *dims, int rad,
                               const float *coef, int ncoef,
                               const float *f0, float *out, int64_t steps,
                               int nthreads)
{
    int64_t px, py, pz;
    if (padded_dims(ndim, dims, rad, ncoef, steps, &px, &py, &pz)) return -1;
    if (nthreads < 1) nthreads = 1;
    size_t n = (size_t)px * (size_t)py * (size_t)pz;
    float *a = (float *)malloc(n * sizeof(float));
    float *b = (float *)malloc(n * sizeof(float));
    if (!a || !b) { free(a); free(b); return -2; }
    memcpy(a, f0, n * sizeof(float));
    for (int64_t t = 0; t < steps; ++t) {
        step_padded_f32(ndim, px, py, pz, rad, coef, a, b, nthreads);
        float *tmp = a; a = b; b = tmp;
    }
    memcpy(out, a, n * sizeof(float));
    free(a);
    free(b);
    return 0;
}

/*
 * Shared-coefficient (symmetric) star, single precision, clamp boundary.
 * Sec. IV.A notes that the paper's instance shares one coefficient per
 * direction while its design targets the case where all coefficients
 * differ; the comparison codes of Sec. VI.C use shared coefficients.  Here
 * the two neighbours at distance i along one axis share one coefficient:
 * coef holds 1 + ndim*rad values, c_C then for i = 1..rad the axes x, y(, z).
 * Each cell is evaluated in this fixed order, one rounding per operation:
 *   acc = c_C * f_C
 *   for i = 1..rad, for each axis a in x, y(, z):
 *       s   = f(p - i e_a) + f(p + i e_a)          (the pair's sum)
 *       acc = fmaf(c_{a,i}, s, acc)
 * In exact arithmetic this is Eq. (1) with c_W,i = c_E,i = c_x,i and so on;
 * the FP64 definition is therefore oracle_star_run_f64 with the
 * coefficients expanded per point.
 */
static void step_sym_f32(int ndim, int64_t nx, int64_t ny, int64_t nz, int rad,
                         const float *c, const float *src, float *dst, int nthreads)
{
#pragma omp parallel for collapse(2) schedule(static) num_threads(nthreads)
    for (int64_t z = 0; z < nz; ++z) {
        for (int64_t y = 0; y < ny; ++y) {
            for (int64_t x = 0; x < nx; ++x) {
#define F(xx, yy, zz) src[(xx) + nx * ((yy) + ny * (zz))]
                float acc = c[0] * F(x, y, z);
                int k = 1;
                for (int i = 1; i <= rad; ++i) {
                    float s = F(clamp_index(x - i, nx), y, z) + F(clamp_index(x + i, nx), y, z);
                    acc = fmaf(c[k], s, acc); ++k;
                    s = F(x, clamp_index(y - i, ny), z) + F(x, clamp_index(y + i, ny), z);
                    acc = fmaf(c[k], s, acc); ++k;
                    if (ndim == 3) {
                        s = F(x, y, clamp_index(z - i, nz)) + F(x, y, clamp_index(z + i, nz));
                        acc = fmaf(c[k], s, acc); ++k;
                    }
                }
                dst[x + nx * (y + ny * z)] = acc;
#undef F
            }
        }
    }
}

int oracle_star_run_sym_f32(int ndim, const int64_t *dims, int rad,
                            const float *coef, int ncoef,
                            const float *f0, float *out, int64_t steps,
                            int nthreads)
{
    int64_t nx, ny, nz;
    /* check_args counts per-point coefficients: pass that count */
    if (ncoef != 1 + ndim * rad) return -1;
    if (check_args(ndim, dims, rad, 1 + 2 * ndim * rad, steps, &nx, &ny, &nz)) return -1;
    if (nthreads < 1) nthreads = 1;
    size_t n = (size_t)nx * (size_t)ny * (size_t)nz;
    float *a = (float *)malloc(n * sizeof(float));
    float *b = (float *)malloc(n * sizeof(float));
    if (!a || !b) { free(a); free(b); return -2; }
    memcpy(a, f0, n * sizeof(float));
    for (int64_t t = 0; t < steps; ++t) {
        step_sym_f32(ndim, nx, ny, nz, rad, coef, a, b, nthreads);
        float *tmp = a; a = b; b = tmp;
    }
    memcpy(out, a, n * sizeof(float));
    free(a);
    free(b);
    return 0;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
