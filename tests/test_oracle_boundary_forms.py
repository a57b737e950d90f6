"""Pins of the oracle's padded-halo boundary and shared-coefficient forms.

Padded halo (Sec. IV.B: YASK allocates a larger grid and reads the
out-of-bound neighbours from memory): the array holds the interior inside a
fixed ghost frame of `radius` cells; each step applies Eq. (1) to the
interior without clamping and keeps the frame.  Pinned against numpy slicing
(pure shifts), a dense affine map built from the definition, the clamp
oracle (one step from an edge-replicated frame), and invariants.

Shared coefficients (Sec. IV.A: one coefficient per direction in the
paper's instance; Sec. VI.C: the comparison codes share coefficients): both
neighbours of an axis and distance share c_{a,i}; the FP32 order is c_C*f_C,
then per distance and axis one fused multiply-add of c_{a,i} with the
rounded pair sum.  Pinned by exact rational arithmetic in that order, by
the FP64 definition with the coefficients expanded per point, and by
expand_symmetric written out by hand.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_2002_05983_amd import synth
from test_oracle_fp32_order import exact, round_binary32

DIRS = {2: "WESN", 3: "WESNBA"}
AXIS = {"W": -1, "E": -1, "S": -2, "N": -2, "B": -3, "A": -3}
SIGN = {"W": -1, "E": 1, "S": -1, "N": 1, "B": -1, "A": 1}


def interior(a, r):
    return a[tuple(slice(r, n - r) for n in a.shape)]


def frame_mask(shape, r):
    m = np.ones(shape, dtype=bool)
    m[tuple(slice(r, n - r) for n in shape)] = False
    return m


# --- padded halo ---------------------------------------------------------------

PADDED_CASES = [((9, 11), 1), ((12, 10), 2), ((9, 14), 4), ((7, 8, 9), 1), ((9, 10, 11), 3),
                ((10, 9, 12), 4)]


@pytest.mark.parametrize("padded,radius", PADDED_CASES)
def test_padded_pure_shift_is_array_slicing(oracle_mod, padded, radius):
    """One coefficient 1 at (d, i), all others 0: the interior becomes the
    padded array shifted by i along d (a plain slice), the frame stays."""
    ndim = len(padded)
    f = synth.grid_uniform(61, padded)
    for i in range(1, radius + 1):
        for d in DIRS[ndim]:
            c = np.zeros(1 + 2 * ndim * radius, dtype=np.float32)
            c[1 + (i - 1) * 2 * ndim + DIRS[ndim].index(d)] = 1.0
            want = f.copy()
            sl = [slice(radius, n - radius) for n in padded]
            src = list(sl)
            ax = AXIS[d]
            src[ax] = slice(radius + SIGN[d] * i, padded[ax] - radius + SIGN[d] * i)
            want[tuple(sl)] = f[tuple(src)]
            for dt in (np.float64, np.float32):
                got = oracle_mod.star_run_padded(f, c, radius, 1, dtype=dt)
                np.testing.assert_array_equal(got, want.astype(dt), err_msg=f"{d}{i}")


def dense_padded_operator(shape, coeffs, radius):
    """Matrix of one padded-halo step over the flattened padded array, built
    from the definition: identity rows for the frame, Eq. (1) rows inside."""
    ndim = len(shape)
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    frame = frame_mask(shape, radius)
    for idx in np.ndindex(*shape):
        row = np.ravel_multi_index(idx, shape)
        if frame[idx]:
            A[row, row] = 1.0
            continue
        A[row, row] += coeffs[0]
        for i in range(1, radius + 1):
            for k, d in enumerate(DIRS[ndim]):
                nb = list(idx)
                nb[AXIS[d]] += SIGN[d] * i
                A[row, np.ravel_multi_index(tuple(nb), shape)] += coeffs[1 + (i - 1) * 2 * ndim + k]
    return A


@pytest.mark.parametrize("padded,radius", [((6, 7), 1), ((8, 9), 2), ((9, 10), 4), ((5, 6, 7), 1),
                                           ((7, 8, 7), 2)])
def test_padded_dense_operator_power(oracle_mod, padded, radius):
    ndim = len(padded)
    c = synth.coefficients(62 + radius, ndim, radius)
    f = synth.grid_uniform(63, padded)
    A = dense_padded_operator(padded, c.astype(np.float64), radius)
    steps = 5
    want = np.linalg.matrix_power(A, steps) @ f.astype(np.float64).ravel()
    got = oracle_mod.star_run_padded(f, c, radius, steps)
    np.testing.assert_allclose(got.ravel(), want, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("padded,radius", PADDED_CASES)
def test_padded_one_step_from_replicated_frame_is_clamp(oracle_mod, padded, radius):
    """With the frame filled by repeating the interior's border cells, one
    padded step reads exactly what the clamp reads: the interiors agree bit
    for bit, in FP64 and in the FP32 order."""
    ndim = len(padded)
    inner = synth.grid_uniform(64, tuple(n - 2 * radius for n in padded))
    f = np.pad(inner, radius, mode="edge")
    c = synth.coefficients(65 + radius, ndim, radius)
    np.testing.assert_array_equal(interior(oracle_mod.star_run_padded(f, c, radius, 1), radius),
                                  oracle_mod.star_run_f64(inner, c, radius, 1))
    np.testing.assert_array_equal(
        interior(oracle_mod.star_run_padded(f, c, radius, 1, dtype=np.float32), radius),
        oracle_mod.star_run_f32(inner, c, radius, 1))
    # after two steps they differ in general: the frame does not follow the border
    two = interior(oracle_mod.star_run_padded(f, c, radius, 2), radius)
    assert not np.array_equal(two, oracle_mod.star_run_f64(inner, c, radius, 2))


@pytest.mark.parametrize("padded,radius", PADDED_CASES)
def test_padded_frame_fixed_and_invariants(oracle_mod, padded, radius):
    ndim = len(padded)
    c = synth.coefficients(66 + radius, ndim, radius)
    f = synth.grid_uniform(67, padded)
    m = frame_mask(padded, radius)
    for dt in (np.float64, np.float32):
        out = oracle_mod.star_run_padded(f, c, radius, 6, dtype=dt)
        np.testing.assert_array_equal(out[m], f[m].astype(dt))
        # step composition, bit for bit
        part = oracle_mod.star_run_padded(oracle_mod.star_run_padded(f, c, radius, 2, dtype=dt),
                                          c, radius, 4, dtype=dt)
        np.testing.assert_array_equal(out, part)
        # max principle: positive coefficients summing to 1
        assert out.min() >= f.min() - 1e-6 and out.max() <= f.max() + 1e-6
    # a dyadic constant field with dyadic coefficients summing to 1 stays fixed
    w = np.ones(1 + 2 * ndim * radius)
    w[0] += 64 - w.sum()
    cd = (w / 64).astype(np.float32)
    k = np.full(padded, 0.375, dtype=np.float32)
    np.testing.assert_array_equal(oracle_mod.star_run_padded(k, cd, radius, 9, dtype=np.float32), k)
    with pytest.raises(ValueError):
        oracle_mod.star_run_padded(np.zeros((2 * radius, 9), np.float32),
                                   synth.coefficients(1, 2, radius), radius, 1)


# --- shared coefficients ---------------------------------------------------------

def test_expand_symmetric_by_hand(oracle_mod):
    sym = np.array([0.5, 0.1, 0.2, 0.01, 0.02], dtype=np.float32)  # 2D, R = 2
    np.testing.assert_array_equal(
        oracle_mod.expand_symmetric(sym, 2, 2),
        np.array([0.5, 0.1, 0.1, 0.2, 0.2, 0.01, 0.01, 0.02, 0.02], dtype=np.float32))
    sym3 = np.array([1, 2, 3, 4], dtype=np.float32)  # 3D, R = 1: x, y, z
    np.testing.assert_array_equal(oracle_mod.expand_symmetric(sym3, 3, 1),
                                  np.array([1, 2, 2, 3, 3, 4, 4], dtype=np.float32))


def sym_step_exact(f, c, radius, pair_rounded=True):
    """One shared-coefficient step, exact arithmetic with one binary32
    rounding per operation, in the order of star_run_sym_f32."""
    ndim = f.ndim
    shape = f.shape
    cf = [exact(v) for v in c]
    out = np.empty_like(f)
    for idx in np.ndindex(*shape):
        acc = round_binary32(cf[0] * exact(f[idx]))
        k = 1
        for i in range(1, radius + 1):
            for ax in range(ndim):  # x, y, z
                a = ndim - 1 - ax
                lo, hi = list(idx), list(idx)
                lo[a] = max(idx[a] - i, 0)
                hi[a] = min(idx[a] + i, shape[a] - 1)
                s = exact(f[tuple(lo)]) + exact(f[tuple(hi)])
                if pair_rounded:
                    s = round_binary32(s)
                acc = round_binary32(cf[k] * s + acc)
                k += 1
        out[idx] = np.float32(float(acc))
    return out


def sym_inputs(shape, radius, seed):
    rng = np.random.default_rng(seed)
    f = (rng.uniform(0.25, 4.0, size=shape) * rng.choice([-1.0, 1.0], size=shape)).astype(np.float32)
    w = rng.uniform(1.0, 2.0, size=1 + len(shape) * radius)
    return f, (w / w.sum()).astype(np.float32)


@pytest.mark.parametrize("shape,radius,steps", [((6, 7), 1, 2), ((5, 9), 3, 1), ((4, 5, 3), 2, 2),
                                                ((3, 4, 5), 4, 1)])
def test_sym_f32_matches_exact_order(oracle_mod, shape, radius, steps):
    f, c = sym_inputs(shape, radius, 70 + radius)
    want = f
    for _ in range(steps):
        want = sym_step_exact(want, c, radius)
    got = oracle_mod.star_run_sym_f32(f, c, radius, steps)
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("shape,radius", [((6, 7), 1), ((4, 5, 3), 2)])
def test_sym_order_is_distinguishable(oracle_mod, shape, radius):
    """The inputs tell the orders apart: the per-point order (two fused
    multiply-adds per pair) and an unrounded pair sum both change bits."""
    f, c = sym_inputs(shape, radius, 70 + radius)
    ref = sym_step_exact(f, c, radius)
    per_point = oracle_mod.star_run_f32(f, oracle_mod.expand_symmetric(c, len(shape), radius),
                                        radius, 1)
    assert np.any(ref.view(np.uint32) != per_point.view(np.uint32))
    unrounded = sym_step_exact(f, c, radius, pair_rounded=False)
    assert np.any(ref.view(np.uint32) != unrounded.view(np.uint32))


@pytest.mark.parametrize("shape,radius", [((64, 70), 1), ((40, 50), 4), ((20, 24, 28), 2),
                                          ((16, 18, 20), 4)])
def test_sym_f32_close_to_fp64_definition(oracle_mod, shape, radius):
    ndim = len(shape)
    w = 1.0 + synth.uniform01_f64(80 + radius, 1 + ndim * radius)
    w[1:] *= 2  # each shared value stands for two points
    sym = (w / w.sum()).astype(np.float32)
    sym[0] = np.float32(1.0) - np.float32(2 * sym[1:].astype(np.float64).sum())
    f = synth.grid_uniform(81, shape)
    steps = 30
    got = oracle_mod.star_run_sym_f32(f, sym, radius, steps)
    ref = oracle_mod.star_run_f64(f, oracle_mod.expand_symmetric(sym, ndim, radius), radius, steps)
    err = oracle_mod.rel_linf(got, ref)
    assert 0 < err <= steps * (1 + 2 * ndim * radius) * 2.0 ** -24
