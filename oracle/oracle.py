"""CPU oracle for star-stencil sweeps -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this module.  The GPU library never does, and this
module imports nothing from the library.

Paper: Zohouri, Podobas, Matsuoka, "High-Performance High-Order Stencil
Computation on FPGAs Using OpenCL" (IPDPSW 2018).

Contents, each with the passage it follows:
  * star_run_f64 / star_run_f32 / star_sample_f64 -- Eq. (1) of Sec. IV.A
    with the clamp-to-border boundary of Sec. III.B / IV.B (C code in
    star_oracle.c).
  * star_run_padded -- the padded-halo boundary of Sec. IV.B (YASK's larger
    allocation: a fixed ghost frame read without clamping).
  * star_run_sym_f32, expand_symmetric -- shared coefficients per axis and
    distance (Sec. IV.A, Sec. VI.C), in a fixed FP32 order.
  * flop_per_cell, bytes_per_cell -- Table I (Sec. IV.A): 8r+1 / 12r+1 FLOP
    and 8 bytes per cell update under full spatial reuse.
  * gcells_per_s, gflops, gbytes_per_s, roofline_ratio -- Eq. (3) (Sec.
    IV.C) read as cells*iterations/time, the derived GFLOP/s and GB/s of the
    same passage, and the roofline ratio of Sec. VI.B.
  * rel_linf, reduce_f64 -- normwise relative L-infinity error and the
    conservation sum, written out from their definitions in FP64.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle_star.so")
_lib = None


def lib() -> ctypes.CDLL:
    """The compiled oracle (built by oracle/build.py)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _build  # local build of the C oracle only
            _build.build()
        L = ctypes.CDLL(_LIB_PATH)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        fp = ctypes.POINTER(ctypes.c_float)
        L.oracle_star_run_f64.argtypes = [ctypes.c_int, i64p, ctypes.c_int, dp, ctypes.c_int,
                                          dp, dp, ctypes.c_int64, ctypes.c_int]
        L.oracle_star_run_f32.argtypes = [ctypes.c_int, i64p, ctypes.c_int, fp, ctypes.c_int,
                                          fp, fp, ctypes.c_int64, ctypes.c_int]
        L.oracle_star_sample_f64.argtypes = [ctypes.c_int, i64p, ctypes.c_int, dp, ctypes.c_int,
                                             fp, ctypes.c_int64, i64p, ctypes.c_int64, dp,
                                             ctypes.c_int]
        L.oracle_star_sample_f32.argtypes = [ctypes.c_int, i64p, ctypes.c_int, fp, ctypes.c_int,
                                             fp, ctypes.c_int64, i64p, ctypes.c_int64, fp,
                                             ctypes.c_int]
        L.oracle_star_run_padded_f64.argtypes = L.oracle_star_run_f64.argtypes
        L.oracle_star_run_padded_f32.argtypes = L.oracle_star_run_f32.argtypes
        L.oracle_star_run_sym_f32.argtypes = L.oracle_star_run_f32.argtypes
        for f in (L.oracle_star_run_f64, L.oracle_star_run_f32, L.oracle_star_sample_f64,
                  L.oracle_star_sample_f32, L.oracle_star_run_padded_f64,
                  L.oracle_star_run_padded_f32, L.oracle_star_run_sym_f32):
            f.restype = ctypes.c_int
        L.oracle_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def _dims_xyz(shape) -> np.ndarray:
    """numpy shape (slowest first) -> dims in x, y[, z] order."""
    return np.ascontiguousarray(np.array(shape[::-1], dtype=np.int64))


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _check(rc: int, what: str):
    if rc == -1:
        raise ValueError(f"{what}: invalid arguments")
    if rc == -2:
        raise MemoryError(f"{what}: out of host memory")
    if rc != 0:
        raise RuntimeError(f"{what}: status {rc}")


def star_run_f64(f0: np.ndarray, coeffs, radius: int, steps: int, threads: int = 0) -> np.ndarray:
    """f^steps by Eq. (1) with clamp, in FP64.

    f0: array of shape (ny, nx) or (nz, ny, nx), promoted exactly to FP64.
    coeffs: 1 + 2*ndim*radius per-point values in canonical order (centre,
    then W,E,S,N[,B,A] for i = 1..radius); FP32 values are promoted exactly.
    """
    f = np.ascontiguousarray(f0, dtype=np.float64)
    c = np.ascontiguousarray(np.asarray(coeffs), dtype=np.float64)
    ndim = f.ndim
    out = np.empty_like(f)
    dims = _dims_xyz(f.shape)
    rc = lib().oracle_star_run_f64(ndim, _ptr(dims, ctypes.c_int64), int(radius),
                                   _ptr(c, ctypes.c_double), int(c.size),
                                   _ptr(f, ctypes.c_double), _ptr(out, ctypes.c_double),
                                   int(steps), int(threads or max_threads()))
    _check(rc, "star_run_f64")
    return out


def star_run_f32(f0: np.ndarray, coeffs, radius: int, steps: int, threads: int = 0) -> np.ndarray:
    """Eq. (1) with clamp evaluated in FP32 in the fixed order c_C*f_C then
    one fused multiply-add per neighbour in coefficient order."""
    f = np.ascontiguousarray(f0, dtype=np.float32)
    c = np.ascontiguousarray(np.asarray(coeffs), dtype=np.float32)
    out = np.empty_like(f)
    dims = _dims_xyz(f.shape)
    rc = lib().oracle_star_run_f32(f.ndim, _ptr(dims, ctypes.c_int64), int(radius),
                                   _ptr(c, ctypes.c_float), int(c.size),
                                   _ptr(f, ctypes.c_float), _ptr(out, ctypes.c_float),
                                   int(steps), int(threads or max_threads()))
    _check(rc, "star_run_f32")
    return out


def star_sample_f64(f0: np.ndarray, coeffs, radius: int, steps: int, cells,
                    threads: int = 0) -> np.ndarray:
    """f^steps (FP64) at the given cells, each from its own dependence cone.

    cells: integer array (n, ndim) of coordinates in x, y[, z] order.
    """
    f = np.ascontiguousarray(f0, dtype=np.float32)
    c = np.ascontiguousarray(np.asarray(coeffs), dtype=np.float64)
    cl = np.asarray(cells, dtype=np.int64)
    tri = np.zeros((cl.shape[0], 3), dtype=np.int64)
    tri[:, :cl.shape[1]] = cl
    tri = np.ascontiguousarray(tri)
    vals = np.empty(cl.shape[0], dtype=np.float64)
    dims = _dims_xyz(f.shape)
    rc = lib().oracle_star_sample_f64(f.ndim, _ptr(dims, ctypes.c_int64), int(radius),
                                      _ptr(c, ctypes.c_double), int(c.size),
                                      _ptr(f, ctypes.c_float), int(steps),
                                      _ptr(tri, ctypes.c_int64), int(cl.shape[0]),
                                      _ptr(vals, ctypes.c_double), int(threads or max_threads()))
    _check(rc, "star_sample_f64")
    return vals


def star_sample_f32(f0: np.ndarray, coeffs, radius: int, steps: int, cells,
                    threads: int = 0) -> np.ndarray:
    """f^steps at the given cells in the FP32 order of star_run_f32, each
    from its own dependence cone (bitwise the full-grid FP32 values).

    cells: integer array (n, ndim) of coordinates in x, y[, z] order.
    """
    f = np.ascontiguousarray(f0, dtype=np.float32)
    c = np.ascontiguousarray(np.asarray(coeffs), dtype=np.float32)
    cl = np.asarray(cells, dtype=np.int64)
    tri = np.zeros((cl.shape[0], 3), dtype=np.int64)
    tri[:, :cl.shape[1]] = cl
    tri = np.ascontiguousarray(tri)
    vals = np.empty(cl.shape[0], dtype=np.float32)
    dims = _dims_xyz(f.shape)
    rc = lib().oracle_star_sample_f32(f.ndim, _ptr(dims, ctypes.c_int64), int(radius),
                                      _ptr(c, ctypes.c_float), int(c.size),
                                      _ptr(f, ctypes.c_float), int(steps),
                                      _ptr(tri, ctypes.c_int64), int(cl.shape[0]),
                                      _ptr(vals, ctypes.c_float), int(threads or max_threads()))
    _check(rc, "star_sample_f32")
    return vals


def star_run_padded(f0: np.ndarray, coeffs, radius: int, steps: int, dtype=np.float64,
                    threads: int = 0) -> np.ndarray:
    """The padded-halo boundary (Sec. IV.B): f0 is the padded array, the
    interior surrounded by a fixed ghost frame of `radius` cells on every
    side; every step applies Eq. (1) to the interior cells, reading
    neighbours from the array without clamping, and keeps the frame.
    dtype float64 (the definition) or float32 (the FP32 order of
    star_run_f32)."""
    f = np.ascontiguousarray(f0, dtype=dtype)
    ct = ctypes.c_double if dtype == np.float64 else ctypes.c_float
    c = np.ascontiguousarray(np.asarray(coeffs), dtype=dtype)
    if any(n <= 2 * radius for n in f.shape):
        raise ValueError("star_run_padded: every axis needs an interior (side > 2*radius)")
    out = np.empty_like(f)
    dims = _dims_xyz(tuple(n - 2 * radius for n in f.shape))
    fn = lib().oracle_star_run_padded_f64 if dtype == np.float64 else lib().oracle_star_run_padded_f32
    rc = fn(f.ndim, _ptr(dims, ctypes.c_int64), int(radius), _ptr(c, ct), int(c.size),
            _ptr(f, ct), _ptr(out, ct), int(steps), int(threads or max_threads()))
    _check(rc, "star_run_padded")
    return out


def expand_symmetric(sym, ndim: int, radius: int) -> np.ndarray:
    """Per-point coefficients of a shared-coefficient star: sym holds c_C,
    then for i = 1..radius one value per axis (x, y[, z]); both neighbours of
    an axis and distance take it (W, E <- x; S, N <- y; B, A <- z)."""
    sym = np.asarray(sym)
    out = [sym[0]]
    for i in range(radius):
        for a in range(ndim):
            v = sym[1 + i * ndim + a]
            out += [v, v]
    return np.array(out, dtype=sym.dtype)


def star_run_sym_f32(f0: np.ndarray, sym_coeffs, radius: int, steps: int,
                     threads: int = 0) -> np.ndarray:
    """Shared-coefficient star in FP32 (clamp boundary): per cell c_C*f_C,
    then for i = 1..radius and each axis one fused multiply-add of c_{a,i}
    with the rounded pair sum f(p - i e_a) + f(p + i e_a).  Its FP64
    definition is star_run_f64 with expand_symmetric(sym_coeffs)."""
    f = np.ascontiguousarray(f0, dtype=np.float32)
    c = np.ascontiguousarray(np.asarray(sym_coeffs), dtype=np.float32)
    out = np.empty_like(f)
    dims = _dims_xyz(f.shape)
    rc = lib().oracle_star_run_sym_f32(f.ndim, _ptr(dims, ctypes.c_int64), int(radius),
                                       _ptr(c, ctypes.c_float), int(c.size),
                                       _ptr(f, ctypes.c_float), _ptr(out, ctypes.c_float),
                                       int(steps), int(threads or max_threads()))
    _check(rc, "star_run_sym_f32")
    return out


# --- Table I and Eq. (3): work and throughput accounting -------------------

def flop_per_cell(ndim: int, radius: int) -> int:
    """Table I: 8r+1 (2D) or 12r+1 (3D) FLOP per cell update -- one multiply
    per point and one add per neighbour (Sec. IV.A)."""
    points = 1 + 2 * ndim * radius
    return points + (points - 1)


def bytes_per_cell(elem_bytes: int = 4) -> int:
    """Table I: one read and one write per cell update under full reuse."""
    return 2 * elem_bytes


def gcells_per_s(cells: float, iterations: float, seconds: float) -> float:
    """Eq. (3), read as cells * iterations / run time, in units of 1e9."""
    return cells * iterations / seconds / 1e9


def gflops(gcells: float, ndim: int, radius: int) -> float:
    """Sec. IV.C: GFLOP/s = GCell/s x FLOP per cell update."""
    return gcells * flop_per_cell(ndim, radius)


def gbytes_per_s(gcells: float, elem_bytes: int = 4) -> float:
    """Sec. IV.C: GB/s = GCell/s x bytes per cell update."""
    return gcells * bytes_per_cell(elem_bytes)


def roofline_ratio(gbs: float, peak_gbs: float) -> float:
    """Sec. VI.B: achieved GB/s over the device's peak memory bandwidth."""
    return gbs / peak_gbs


# --- error norm and conservation sum ---------------------------------------

def reduce_f64(x: np.ndarray, ref: np.ndarray):
    """(max|x - ref|, max|ref|, sum x), all in FP64."""
    xd = np.asarray(x, dtype=np.float64).ravel()
    rd = np.asarray(ref, dtype=np.float64).ravel()
    return float(np.max(np.abs(xd - rd))), float(np.max(np.abs(rd))), float(np.sum(xd))


def rel_linf(x: np.ndarray, ref: np.ndarray) -> float:
    """Normwise relative L-infinity error: max|x - ref| / max|ref|."""
    d, m, _ = reduce_f64(x, ref)
    return d / m if m > 0 else d
