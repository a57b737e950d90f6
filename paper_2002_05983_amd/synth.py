"""Seeded synthetic inputs for star-stencil sweeps.

This module only draws numbers: grid values, coefficient sets, grid shapes.
It holds none of the stencil arithmetic, so both the GPU path and the CPU
oracle can be fed from it without sharing any of the method's code.

Random source: SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), used in its counter form:
the i-th draw of stream ``seed`` is ``mix64(seed + (i + 1) * GAMMA)``, with
GAMMA = 0x9E3779B97F4A7C15 and the published 64-bit finaliser
``z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
z *= 0x94D049BB133111EB; z ^= z >> 31``.  The counter form lets any slice
of a stream be produced independently, so large grids are generated in
chunks.

Grid values are ``(draw >> 40) * 2**-24``: multiples of 2**-24 in [0, 1),
exactly representable in FP32, so an FP32 grid and its FP64 promotion hold
the same numbers.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22


def splitmix64(seed: int, start: int, count: int) -> np.ndarray:
    """Draws ``start .. start+count-1`` of SplitMix64 stream ``seed`` (uint64)."""
    with np.errstate(over="ignore"):
        ctr = np.arange(start + 1, start + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + ctr * GAMMA
        z ^= z >> np.uint64(30)
        z *= _M1
        z ^= z >> np.uint64(27)
        z *= _M2
        z ^= z >> np.uint64(31)
    return z


def uniform01_f32(seed: int, count: int, start: int = 0) -> np.ndarray:
    """``count`` FP32 values k * 2**-24, k a 24-bit integer from the stream."""
    out = np.empty(count, dtype=np.float32)
    for lo in range(0, count, _CHUNK):
        n = min(_CHUNK, count - lo)
        k = splitmix64(seed, start + lo, n) >> np.uint64(40)
        out[lo:lo + n] = k.astype(np.float32) * np.float32(2.0 ** -24)
    return out


def uniform01_f64(seed: int, count: int, start: int = 0) -> np.ndarray:
    """``count`` FP64 values in [0, 1) with 53 random bits (for shape draws)."""
    k = splitmix64(seed, start, count) >> np.uint64(11)
    return k.astype(np.float64) * 2.0 ** -53


def grid_uniform(seed: int, shape) -> np.ndarray:
    """A C-ordered FP32 grid (slowest axis first) with values U[0,1) from seed."""
    n = int(np.prod(shape))
    return uniform01_f32(seed, n).reshape(shape)


def num_points(ndim: int, radius: int) -> int:
    """Points of a star stencil: the centre plus 2*ndim*radius axis neighbours."""
    return 1 + 2 * ndim * radius


def coefficients(seed: int, ndim: int, radius: int) -> np.ndarray:
    """Seeded positive per-point FP32 coefficients that sum to 1 (up to FP32).

    w_j = 1 + U[0,1) per point, c_j = fl32(w_j / sum(w)) with the division in
    FP64.  All coefficients are within a factor of two of each other.  The
    order of the points is the library's canonical one: centre, then for each
    distance i = 1..radius the directions W, E, S, N (and B, A in 3D).
    """
    p = num_points(ndim, radius)
    w = 1.0 + uniform01_f64(seed, p)
    return (w / w.sum()).astype(np.float32)


def sinusoid_grid(seed: int, n: int, modes: int = 8, noise: float = 1e-3,
                  kmax: int = 3) -> np.ndarray:
    """A cube of side n: a seeded sum of low-frequency sinusoids plus noise.

    f(x,y,z) = sum_j a_j sin(2 pi (kx_j x + ky_j y + kz_j z) / n + phi_j)
               + noise * U[0,1)
    with a_j ~ U[0.5,1), integer k per axis in [0, kmax] (not all zero) and
    phi_j ~ U[0, 2 pi).  Evaluated in FP64 (each mode split by the angle
    addition formula into an xy factor and a z factor), rounded to FP32.
    """
    draws = uniform01_f64(seed, 16 * modes)
    amp, kvec, phase = [], [], []
    for j in range(modes):
        d = draws[16 * j:16 * j + 16]
        amp.append(0.5 + 0.5 * d[0])
        k = [int(d[1 + a] * (kmax + 1)) for a in range(3)]
        t = 4
        while k == [0, 0, 0]:
            k = [int(d[t + a] * (kmax + 1)) for a in range(3)]
            t += 3
            if t + 3 > 16:
                k = [1, 0, 0]
        kvec.append(k)
        phase.append(2.0 * math.pi * d[15])
    # sin(t_xy + t_z) = sin(t_xy) cos(t_z) + cos(t_xy) sin(t_z): the field is
    # a (planes x 2*modes) by (2*modes x cells-per-plane) matrix product.
    ax = np.arange(n, dtype=np.float64)
    yy, xx = np.meshgrid(ax, ax, indexing="ij")
    basis = np.empty((2 * modes, n * n), dtype=np.float64)
    for j, (k, ph) in enumerate(zip(kvec, phase)):
        t_xy = (2.0 * math.pi * (k[0] * xx + k[1] * yy) / n + ph).ravel()
        basis[2 * j] = np.sin(t_xy)
        basis[2 * j + 1] = np.cos(t_xy)
    out = np.empty((n, n, n), dtype=np.float32)
    zc = max(1, (1 << 22) // (n * n))  # planes per chunk
    for z0 in range(0, n, zc):
        z = np.arange(z0, min(n, z0 + zc), dtype=np.float64)
        w = np.empty((z.size, 2 * modes), dtype=np.float64)
        for j, (a, k) in enumerate(zip(amp, kvec)):
            t_z = 2.0 * math.pi * k[2] * z / n
            w[:, 2 * j] = a * np.cos(t_z)
            w[:, 2 * j + 1] = a * np.sin(t_z)
        vals = w @ basis
        noise_vals = uniform01_f32(seed + 1, z.size * n * n, start=z0 * n * n).astype(np.float64)
        out[z0:z0 + z.size] = (vals + noise * noise_vals.reshape(z.size, n * n)).reshape(
            z.size, n, n).astype(np.float32)
    return out


def batch_shapes(seed: int, n2d: int = 128, n3d: int = 128, lo2: int = 64, hi2: int = 4096,
                 lo3: int = 32, hi3: int = 256):
    """Shapes and radii of a mixed batch of grids.

    Each side is drawn independently, log-uniform in [lo, hi] and rounded to
    an integer; the radius is uniform in 1..4.  Returns a list of
    (dims tuple in x, y[, z] order, radius, coefficient seed, value seed).
    """
    count = n2d + n3d
    d = uniform01_f64(seed, 8 * count)
    out = []
    for g in range(count):
        u = d[8 * g:8 * g + 8]
        if g < n2d:
            nd, lo, hi = 2, lo2, hi2
        else:
            nd, lo, hi = 3, lo3, hi3
        dims = tuple(int(round(math.exp(math.log(lo) + u[a] * (math.log(hi) - math.log(lo)))))
                     for a in range(nd))
        radius = 1 + min(3, int(u[3] * 4))
        out.append((dims, radius, seed * 1000 + 2 * g + 1, seed * 1000 + 2 * g + 2))
    return out
