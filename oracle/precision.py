"""CPU model of the precision form -- TEST INFRASTRUCTURE ONLY.

The paper computes in FP32 only (Sec. IV.C); the library adds a form that
stores the state in FP16 or BF16 with one power-of-two scale per 64^3 tile
and does all arithmetic in FP32.  Its result is an approximation, so this
model follows the algorithm's steps in order, in plain numpy, on top of
the oracle's single-precision step (Eq. (1) with clamp, fixed operation
order):

  F = A + D: A is an FP32 anchor, D a scaled low-precision delta.
  For each window of m steps (the last may be shorter):
    G   = fl32(S A - A)                      S = one step of Eq. (1)
    eG  = tile exponents of max|G| per tile; G16 = encode(G)
    D   = G16,  MD = max|G| per tile
    repeat (window - 1) times:
      e   = tile exponents of  s1 * max_{27 neighbour tiles} MD
                               + max|G|,   s1 = sum_k |c_k|
      V   = fl32(S dec(D) + dec(G16)),  MD = max|V| per tile
      D   = encode(V, e)
    A = fl32(A + dec(D))
  result = A
(the maxima are taken before rounding to codes)

The scaled-state form (a second reading of the same storage) keeps the
state itself as codes between FP32 anchor steps:

  For each window of m steps (the last may be shorter):
    eQ = tile exponents of max|A| per tile;  Q = encode(A, eQ);  MQ = max|A|
    repeat (window - 1) times:
      e   = tile exponents of  s1 * max_{27 neighbour tiles} MQ
      V   = fl32(S dec(Q)),  MQ = max|V| per tile
      Q   = encode(V, e)
    A = fl32(S dec(Q))                       one FP32 step (the anchor)
  result = A

Codes: value = q * 2^e.  Encoding scales by 2^-e (exact) and rounds to the
nearest code, ties to even (IEEE binary16 via numpy, bfloat16 by the same
rule on the top 16 bits of the binary32 pattern).  Tile exponent for a
bound B: ceil(log2 B) - 14, or 0 when B = 0.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle

TILE = 64
HEADROOM_BITS = 14
F16, BF16 = 1, 2


def f16_encode(x32: np.ndarray) -> np.ndarray:
    """binary32 -> binary16 bit patterns, round to nearest, ties to even."""
    return np.asarray(x32, dtype=np.float32).astype(np.float16).view(np.uint16)


def f16_decode(q: np.ndarray) -> np.ndarray:
    return np.asarray(q, dtype=np.uint16).view(np.float16).astype(np.float32)


def bf16_encode(x32: np.ndarray) -> np.ndarray:
    """binary32 -> bfloat16 bit patterns, round to nearest, ties to even
    (finite inputs)."""
    b = np.asarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_decode(q: np.ndarray) -> np.ndarray:
    return (np.asarray(q, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def encode(x32, e, codec):
    s = np.ldexp(np.asarray(x32, dtype=np.float32), -np.asarray(e, dtype=np.int32)).astype(np.float32)
    return f16_encode(s) if codec == F16 else bf16_encode(s)


def decode(q, e, codec):
    v = f16_decode(q) if codec == F16 else bf16_decode(q)
    return np.ldexp(v, np.asarray(e, dtype=np.int32)).astype(np.float32)


def tile_exponent(B: float) -> int:
    """ceil(log2 B) - 14 for B > 0, else 0."""
    if not B > 0.0:
        return 0
    m, k = math.frexp(B)
    return (k - 1 if m == 0.5 else k) - HEADROOM_BITS


def tile_shape(shape):
    return tuple((n + TILE - 1) // TILE for n in shape)


def tile_max(x: np.ndarray) -> np.ndarray:
    """max |x| over each 64^3 tile (array of shape tile_shape)."""
    nz, ny, nx = x.shape
    tz, ty, tx = tile_shape(x.shape)
    pad = np.zeros((tz * TILE, ty * TILE, tx * TILE), dtype=np.float32)
    pad[:nz, :ny, :nx] = np.abs(x)
    return pad.reshape(tz, TILE, ty, TILE, tx, TILE).max(axis=(1, 3, 5))


def per_cell(tab: np.ndarray, shape) -> np.ndarray:
    """Broadcast a per-tile table to cells."""
    nz, ny, nx = shape
    return np.repeat(np.repeat(np.repeat(tab, TILE, 0), TILE, 1), TILE, 2)[:nz, :ny, :nx]


def neighbour_max(tab: np.ndarray) -> np.ndarray:
    """max over the 27-tile neighbourhood (clipped at the tile grid)."""
    p = np.pad(tab, 1, mode="constant", constant_values=0.0)
    out = np.zeros_like(tab)
    tz, ty, tx = tab.shape
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                out = np.maximum(out, p[dz:dz + tz, dy:dy + ty, dx:dx + tx])
    return out


def exponents(bounds: np.ndarray) -> np.ndarray:
    return np.vectorize(tile_exponent, otypes=[np.int32])(bounds.astype(np.float64))


def code_values(v, e):
    """The scaled values v * 2^-e that encoding rounds to codes."""
    return np.ldexp(np.asarray(v, dtype=np.float64), -np.asarray(e, dtype=np.int32))


def run(f0: np.ndarray, coeffs, radius: int, steps: int, m: int, codec: int,
        threads: int = 0, observe=None) -> np.ndarray:
    """The precision form on a 3D FP32 grid; returns the FP32 result.
    observe(kind, scaled), if given, sees the scaled values of every encode
    (kind "G" or "D"); it changes nothing."""
    c32 = np.asarray(coeffs, dtype=np.float32)
    s1 = 0.0
    for v in c32:  # summed in coefficient order, in double
        s1 += abs(float(v))
    A = np.array(f0, dtype=np.float32, copy=True)
    shape = A.shape

    def step(x):
        return oracle.star_run_f32(x, c32, radius, 1, threads)

    t = 0
    while t < steps:
        w = min(m, steps - t)
        G = (step(A) - A).astype(np.float32)
        max_g = tile_max(G)
        eG = exponents(max_g)
        g16 = encode(G, per_cell(eG, shape), codec)
        gdec = decode(g16, per_cell(eG, shape), codec)
        if observe:
            observe("G", code_values(G, per_cell(eG, shape)))
        ddec, max_d = gdec, max_g
        for _ in range(1, w):
            bound = s1 * neighbour_max(max_d).astype(np.float64) + max_g.astype(np.float64)
            e = exponents(bound)
            v = (step(ddec) + gdec).astype(np.float32)
            max_d = tile_max(v)
            if observe:
                observe("D", code_values(v, per_cell(e, shape)))
            ddec = decode(encode(v, per_cell(e, shape), codec), per_cell(e, shape), codec)
        A = (A + ddec).astype(np.float32)
        t += w
    return A


def run_scaled(f0: np.ndarray, coeffs, radius: int, steps: int, m: int, codec: int,
               threads: int = 0, observe=None) -> np.ndarray:
    """The scaled-state form on a 3D FP32 grid; returns the FP32 result.
    observe(kind, scaled), if given, sees the scaled values of every encode
    (kind "Q"); it changes nothing."""
    c32 = np.asarray(coeffs, dtype=np.float32)
    s1 = 0.0
    for v in c32:  # summed in coefficient order, in double
        s1 += abs(float(v))
    A = np.array(f0, dtype=np.float32, copy=True)
    shape = A.shape

    def step(x):
        return oracle.star_run_f32(x, c32, radius, 1, threads)

    t = 0
    while t < steps:
        w = min(m, steps - t)
        max_q = tile_max(A)
        e = exponents(max_q)
        if observe:
            observe("Q", code_values(A, per_cell(e, shape)))
        qdec = decode(encode(A, per_cell(e, shape), codec), per_cell(e, shape), codec)
        for _ in range(1, w):
            bound = s1 * neighbour_max(max_q).astype(np.float64)
            e = exponents(bound)
            v = step(qdec)
            max_q = tile_max(v)
            if observe:
                observe("Q", code_values(v, per_cell(e, shape)))
            qdec = decode(encode(v, per_cell(e, shape), codec), per_cell(e, shape), codec)
        A = step(qdec)
        t += w
    return A
