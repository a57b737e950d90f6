"""Pins the single-precision form of the oracle to its operation order.

The paper forbids reordering the sum of Eq. (1) (Sec. IV.A) and counts one
fused multiply-add per point but the first (Sec. V.A).  The FP32 form
evaluates c_C*f_C rounded once, then for i = 1..R and d = W, E, S, N(, B, A)
one rounding of the exact value c_{d,i}*f_{d,i} + acc.  This file restates
that order with exact rational arithmetic (fractions.Fraction) and a
round-to-nearest-even step to binary32 written from the IEEE 754
definition, and compares both the full-grid sweep (star_run_f32) and the
dependence-cone evaluation (star_sample_f32) with it bit for bit.

Inputs have full 24-bit significands so that rounding decisions differ
between orders.  The test first checks that it can tell orders apart: an
unfused evaluation (product rounded, then sum rounded) and a W/E-swapped
order both give different bits for some cell.
"""
from fractions import Fraction

import numpy as np
import pytest

DIRS = {2: "WESN", 3: "WESNBA"}
OFFSET = {"W": (0, -1), "E": (0, 1), "S": (1, -1), "N": (1, 1), "B": (2, -1), "A": (2, 1)}

_MIN_NORMAL_EXP = -126
_MANT_BITS = 23


def round_binary32(q: Fraction) -> Fraction:
    """The binary32 number nearest to q, ties to the even significand
    (IEEE 754 roundTiesToEven); finite results only."""
    if q == 0:
        return Fraction(0)
    sign = -1 if q < 0 else 1
    a = abs(q)
    # exponent e with 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    assert Fraction(2) ** e <= a < Fraction(2) ** (e + 1)
    e = max(e, _MIN_NORMAL_EXP)                   # subnormals share the least quantum
    quantum = Fraction(2) ** (e - _MANT_BITS)
    m = a / quantum
    n = m.numerator // m.denominator
    rest = m - n
    if rest > Fraction(1, 2) or (rest == Fraction(1, 2) and n % 2 == 1):
        n += 1
    out = sign * n * quantum
    assert abs(out) <= Fraction(2) ** 127 * (2 - Fraction(2) ** -23)
    return out


def exact(v) -> Fraction:
    return Fraction(float(v))


def neighbour_terms(ndim, radius, order="WESNBA"):
    """(coefficient index, direction, distance) in the canonical order, or
    with the directions of each distance visited in `order`."""
    dirs = DIRS[ndim]
    out = []
    for i in range(1, radius + 1):
        for d in [d for d in order if d in dirs]:
            out.append((1 + (i - 1) * 2 * ndim + dirs.index(d), d, i))
    return out


def step_exact(f, c, radius, fused=True, order="WESNBA"):
    """One step of Eq. (1) with clamp, each cell evaluated in the stated
    order with one binary32 rounding per operation (fused: one per term)."""
    ndim = f.ndim
    shape = f.shape  # slowest first
    cf = [exact(v) for v in c]
    out = np.empty_like(f)
    terms = neighbour_terms(ndim, radius, order)
    for idx in np.ndindex(*shape):
        xyz = list(idx[::-1])  # x, y(, z)
        acc = round_binary32(cf[0] * exact(f[idx]))
        for k, d, i in terms:
            axis, sign = OFFSET[d]
            p = list(xyz)
            p[axis] = min(max(p[axis] + sign * i, 0), shape[ndim - 1 - axis] - 1)
            val = exact(f[tuple(p[::-1])])
            if fused:
                acc = round_binary32(cf[k] * val + acc)
            else:
                acc = round_binary32(round_binary32(cf[k] * val) + acc)
        out[idx] = np.float32(float(acc))
    return out


def run_exact(f, c, radius, steps, **kw):
    for _ in range(steps):
        f = step_exact(f, c, radius, **kw)
    return f


def full_mantissa_inputs(shape, ndim, radius, seed):
    """Grid values and coefficients with random 24-bit significands."""
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.25, 4.0, size=shape).astype(np.float32)
    f *= rng.choice(np.array([1.0, -1.0], dtype=np.float32), size=shape)
    w = rng.uniform(1.0, 2.0, size=1 + 2 * ndim * radius)
    c = (w / w.sum()).astype(np.float32)
    return f, c


CASES = [((6, 7), 1, 2), ((5, 9), 2, 2), ((4, 3), 4, 1), ((4, 5, 3), 1, 2), ((3, 4, 5), 2, 1),
         ((2, 3, 4), 4, 1)]


@pytest.mark.parametrize("shape,radius,steps", CASES)
def test_f32_sweep_matches_exact_order(oracle_mod, shape, radius, steps):
    ndim = len(shape)
    f, c = full_mantissa_inputs(shape, ndim, radius, seed=7 + radius + 10 * ndim)
    want = run_exact(f, c, radius, steps)
    got = oracle_mod.star_run_f32(f, c, radius, steps)
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))
    dims = shape[::-1]
    cells = np.array([p[::-1] for p in np.ndindex(*shape)], dtype=np.int64)
    vals = oracle_mod.star_sample_f32(f, c, radius, steps, cells)
    np.testing.assert_array_equal(vals.view(np.uint32),
                                  np.array([want[tuple(p[::-1])] for p in cells]).view(np.uint32))
    assert cells.shape[1] == len(dims)


@pytest.mark.parametrize("shape,radius", [((6, 7), 1), ((5, 9), 2), ((4, 5, 3), 1)])
def test_exact_order_tells_orders_apart(shape, radius):
    """The inputs are chosen so that the order matters: a plain multiply
    then add, and W before E swapped, each change the bits of some cell."""
    ndim = len(shape)
    f, c = full_mantissa_inputs(shape, ndim, radius, seed=7 + radius + 10 * ndim)
    ref = step_exact(f, c, radius)
    unfused = step_exact(f, c, radius, fused=False)
    swapped = step_exact(f, c, radius, order="EWSNBA")
    assert np.any(ref.view(np.uint32) != unfused.view(np.uint32))
    assert np.any(ref.view(np.uint32) != swapped.view(np.uint32))


def test_round_binary32_against_numpy():
    """The rounding step agrees with the FP64 -> FP32 conversion on exact
    binary64 inputs, including ties and subnormals."""
    rng = np.random.default_rng(3)
    x = np.concatenate([rng.normal(0, 1, 2000), rng.normal(0, 1e-39, 200),
                        rng.uniform(-1e30, 1e30, 200)])
    # exact ties: midpoints of consecutive binary32 numbers
    a = rng.uniform(0.5, 8.0, 200).astype(np.float32)
    b = np.nextafter(a, np.float32(np.inf))
    ties = (a.astype(np.float64) + b.astype(np.float64)) / 2
    x = np.concatenate([x, ties, -ties])
    for v in x:
        assert float(round_binary32(Fraction(float(v)))) == float(np.float32(v)), v
