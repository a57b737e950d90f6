"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: textbook
routines (numpy edge padding, dense matrix powers), closed forms, invariants
and the numbers printed in the paper's tables.  Chosen so that a dropped
term, a wrong sign or distance, a swapped axis or a wrong clamp fails at
least one of them.
"""
import math

import numpy as np
import pytest

from conftest import golden
from paper_2002_05983_amd import synth

DIRS = {2: "WESN", 3: "WESNBA"}


def coef_index(ndim, d, i):
    """Position of neighbour (direction d, distance i) in the per-point order."""
    return 1 + (i - 1) * 2 * ndim + DIRS[ndim].index(d)


def edge_shift(f, d, i):
    """f at the neighbour (d, i) of every cell, clamped -- via numpy edge padding."""
    axis = {"W": -1, "E": -1, "S": -2, "N": -2, "B": -3, "A": -3}[d]
    sign = -1 if d in "WSB" else 1
    pad = [(0, 0)] * f.ndim
    pad[axis] = (i, i)
    g = np.pad(f, pad, mode="edge")
    n = f.shape[axis]
    start = i + sign * i
    sl = [slice(None)] * f.ndim
    sl[axis] = slice(start, start + n)
    return g[tuple(sl)]


def dyadic_coeffs(ndim, radius, symmetric=False, total=64):
    """Coefficients that are multiples of 1/total, positive, summing to 1."""
    p = 1 + 2 * ndim * radius
    w = np.ones(p)
    rem = total - p
    assert rem >= 0
    k = 0
    while rem > 0:
        if symmetric and k > 0:
            # add the same weight to both members of a W/E, S/N, B/A pair
            j = 1 + ((k - 1) % ((p - 1) // 2)) * 2
            if rem >= 2:
                w[j] += 1
                w[j + 1] += 1
                rem -= 2
            else:
                w[0] += 1
                rem -= 1
        else:
            w[k % p] += 1
            rem -= 1
        k += 1
    return (w / total).astype(np.float32)


SHAPES_2D = [(7, 5), (1, 6), (5, 1), (1, 1), (3, 2), (9, 11)]
SHAPES_3D = [(4, 5, 6), (1, 3, 2), (2, 1, 1), (5, 3, 4)]


@pytest.mark.parametrize("radius", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", SHAPES_2D + SHAPES_3D)
def test_pure_shift_matches_edge_padding(oracle_mod, radius, shape):
    """One step with a single unit coefficient is an edge-clamped shift.

    Pins the coefficient order, each direction's axis and sign, the distance
    i, and the clamp of Sec. III.B (out-of-grid neighbours take the border
    cell), including sides smaller than the radius."""
    ndim = len(shape)
    f = synth.grid_uniform(7, shape)
    for i in range(1, radius + 1):
        for d in DIRS[ndim]:
            c = np.zeros(1 + 2 * ndim * radius, dtype=np.float32)
            c[coef_index(ndim, d, i)] = 1.0
            want = edge_shift(f.astype(np.float64), d, i)
            np.testing.assert_array_equal(oracle_mod.star_run_f64(f, c, radius, 1), want)
            np.testing.assert_array_equal(oracle_mod.star_run_f32(f, c, radius, 1),
                                          want.astype(np.float32))
    c = np.zeros(1 + 2 * ndim * radius, dtype=np.float32)
    c[0] = 1.0
    np.testing.assert_array_equal(oracle_mod.star_run_f64(f, c, radius, 3), f)


def dense_operator(shape, ndim, radius, c):
    """The one-step operator as a dense matrix, assembled column by column
    from edge-padded shifts of unit vectors."""
    n = int(np.prod(shape))
    A = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        e = e.reshape(shape)
        col = c[0] * e
        for i in range(1, radius + 1):
            for d in DIRS[ndim]:
                col = col + float(c[coef_index(ndim, d, i)]) * edge_shift(e, d, i)
        A[:, j] = col.ravel()
    return A


@pytest.mark.parametrize("radius", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", [(7, 5), (3, 9), (1, 4), (4, 5, 6), (2, 3, 3)])
def test_brute_force_matrix_power(oracle_mod, radius, shape):
    """oracle(f, s) equals A^s f for the dense operator on tiny grids."""
    ndim = len(shape)
    c = synth.coefficients(100 + radius, ndim, radius).astype(np.float64)
    A = dense_operator(shape, ndim, radius, c)
    f = synth.grid_uniform(3, shape).astype(np.float64)
    for s in (1, 2, 5):
        want = (np.linalg.matrix_power(A, s) @ f.ravel()).reshape(shape)
        got = oracle_mod.star_run_f64(f, c, radius, s)
        np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("radius", [5, 6, 7, 8])
@pytest.mark.parametrize("shape", [(11, 9), (3, 12), (1, 10), (17, 2)])
def test_high_radius_2d_pins(oracle_mod, radius, shape):
    """2D radius 5..8: unit-coefficient shifts equal edge-padded shifts, and
    oracle(f, s) equals A^s f, on grids whose sides are below, at and above
    the radius."""
    f = synth.grid_uniform(9, shape)
    for i in (1, radius - 1, radius):
        for d in DIRS[2]:
            c = np.zeros(1 + 4 * radius, dtype=np.float32)
            c[coef_index(2, d, i)] = 1.0
            want = edge_shift(f.astype(np.float64), d, i)
            np.testing.assert_array_equal(oracle_mod.star_run_f64(f, c, radius, 1), want)
            np.testing.assert_array_equal(oracle_mod.star_run_f32(f, c, radius, 1),
                                          want.astype(np.float32))
    c = synth.coefficients(150 + radius, 2, radius).astype(np.float64)
    A = dense_operator(shape, 2, radius, c)
    g = f.astype(np.float64)
    for s in (1, 3):
        want = (np.linalg.matrix_power(A, s) @ g.ravel()).reshape(shape)
        np.testing.assert_allclose(oracle_mod.star_run_f64(g, c, radius, s), want,
                                   rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("radius", [5, 6, 7, 8])
@pytest.mark.parametrize("shape", [(3, 4, 10), (9, 2, 3), (1, 1, 12)])
def test_high_radius_3d_pins(oracle_mod, radius, shape):
    """3D radius 5..8: unit-coefficient shifts along every axis equal
    edge-padded shifts, and oracle(f, s) equals A^s f on grids whose sides
    are below and above the radius."""
    f = synth.grid_uniform(19, shape)
    for i in (1, radius - 1, radius):
        for d in DIRS[3]:
            c = np.zeros(1 + 6 * radius, dtype=np.float32)
            c[coef_index(3, d, i)] = 1.0
            want = edge_shift(f.astype(np.float64), d, i)
            np.testing.assert_array_equal(oracle_mod.star_run_f64(f, c, radius, 1), want)
            np.testing.assert_array_equal(oracle_mod.star_run_f32(f, c, radius, 1),
                                          want.astype(np.float32))
    c = synth.coefficients(170 + radius, 3, radius).astype(np.float64)
    A = dense_operator(shape, 3, radius, c)
    g = f.astype(np.float64)
    for s in (1, 3):
        want = (np.linalg.matrix_power(A, s) @ g.ravel()).reshape(shape)
        np.testing.assert_allclose(oracle_mod.star_run_f64(g, c, radius, s), want,
                                   rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("shape", [(13, 17), (6, 7, 9)])
def test_linearity(oracle_mod, shape):
    ndim = len(shape)
    for radius in (1, 3):
        c = synth.coefficients(5, ndim, radius)
        f = synth.grid_uniform(11, shape).astype(np.float64)
        g = synth.grid_uniform(12, shape).astype(np.float64)
        a, b = 0.75, -2.5
        lhs = oracle_mod.star_run_f64(a * f + b * g, c, radius, 4)
        rhs = a * oracle_mod.star_run_f64(f, c, radius, 4) + b * oracle_mod.star_run_f64(g, c, radius, 4)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("radius", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", [(8, 9), (1, 1), (2, 7), (5, 4, 3), (1, 1, 2)])
def test_constant_field_is_fixed_bitwise(oracle_mod, radius, shape):
    """With dyadic coefficients summing to exactly 1, a dyadic constant field
    stays fixed bit for bit, at every cell including the border."""
    ndim = len(shape)
    c = dyadic_coeffs(ndim, radius)
    assert float(np.sum(c.astype(np.float64))) == 1.0
    f = np.full(shape, 0.375, dtype=np.float32)
    np.testing.assert_array_equal(oracle_mod.star_run_f64(f, c, radius, 10), f)
    np.testing.assert_array_equal(oracle_mod.star_run_f32(f, c, radius, 10), f)


def test_constant_field_drifts_with_coefficient_sum(oracle_mod):
    """With seeded FP32 coefficients the constant field scales as (sum c)^s."""
    c = synth.coefficients(42, 3, 4)
    s = float(np.sum(c.astype(np.float64)))
    f = np.full((4, 5, 6), 0.5, dtype=np.float32)
    got = oracle_mod.star_run_f64(f, c, 4, 7)
    np.testing.assert_allclose(got, 0.5 * s ** 7, rtol=1e-14)


def _interior(shape, margin):
    sl = []
    for n in shape:
        if n <= 2 * margin:
            return None
        sl.append(slice(margin, n - margin))
    return tuple(sl)


@pytest.mark.parametrize("radius", [1, 2, 3, 4])
@pytest.mark.parametrize("ndim", [2, 3])
def test_polynomials_in_the_interior(oracle_mod, radius, ndim):
    """Symmetric coefficients reproduce degree <= 1 and multilinear fields
    exactly at cells at least s*R from every face; x^2 gains the second
    moment sum_i (c_W,i + c_E,i) i^2 (a negative control that pins the
    distance i and the x axis)."""
    c = dyadic_coeffs(ndim, radius, symmetric=True)
    for i in range(1, radius + 1):
        for a, b in (("W", "E"), ("S", "N"), ("B", "A"))[:ndim]:
            assert c[coef_index(ndim, a, i)] == c[coef_index(ndim, b, i)]
    shape = (24, 26) if ndim == 2 else (13, 14, 15)
    grids = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    x, y = grids[-1], grids[-2]
    z = grids[0] if ndim == 3 else np.zeros(shape)
    fields = [3 + 2 * x - 5 * y + (7 * z if ndim == 3 else 0), x * y, 2 - x * y + 3 * y]
    if ndim == 3:
        fields += [x * z, y * z, x * y * z / 4.0]
    steps = 1 if radius >= 3 else 2
    for f in fields:
        assert np.max(np.abs(f)) < 2 ** 12
        sl = _interior(shape, steps * radius)
        for run in (oracle_mod.star_run_f64, oracle_mod.star_run_f32):
            got = run(f.astype(np.float32), c, radius, steps)
            np.testing.assert_array_equal(got[sl], f.astype(got.dtype)[sl])
    # negative control: x^2 after one step
    f = x * x
    moment = sum(float(c[coef_index(ndim, "W", i)] + c[coef_index(ndim, "E", i)]) * i * i
                 for i in range(1, radius + 1))
    sl = _interior(shape, radius)
    got = oracle_mod.star_run_f64(f.astype(np.float32), c, radius, 1)
    np.testing.assert_array_equal(got[sl], (f + moment)[sl])
    assert moment > 0


@pytest.mark.parametrize("shape,ks", [((10, 12), (1, 3)), ((9, 6, 7), (2, 1, 3)), ((16, 5), (4, 0))])
def test_cosine_eigenvector_radius1(oracle_mod, shape, ks):
    """For radius 1 the clamp is an even reflection about -1/2 and n-1/2, so
    prod_a cos(pi k_a (x_a + 1/2) / n_a) is an exact eigenvector with
    eigenvalue c_C + sum_a 2 c_a cos(pi k_a / n_a) (symmetric coefficients)."""
    ndim = len(shape)
    rng = np.random.default_rng(5)
    ca = rng.uniform(0.05, 0.15, size=ndim)  # per axis, x first
    c = np.zeros(1 + 2 * ndim)
    for a, (lo, hi) in enumerate((("W", "E"), ("S", "N"), ("B", "A"))[:ndim]):
        c[coef_index(ndim, lo, 1)] = ca[a]
        c[coef_index(ndim, hi, 1)] = ca[a]
    c[0] = 1.0 - 2 * ca.sum()
    axes = [np.arange(n, dtype=np.float64) for n in shape]
    grids = np.meshgrid(*axes, indexing="ij")
    f0 = np.ones(shape)
    lam = c[0]
    for a in range(ndim):  # a = 0 is x (last numpy axis)
        n = shape[ndim - 1 - a]
        k = ks[a]
        f0 = f0 * np.cos(math.pi * k * (grids[ndim - 1 - a] + 0.5) / n)
        lam += 2 * ca[a] * math.cos(math.pi * k / n)
    # the oracle promotes its input from FP64 exactly when given FP64
    for s in (1, 3, 8):
        got = oracle_mod.star_run_f64(f0, c, 1, s)
        np.testing.assert_allclose(got, lam ** s * f0, rtol=0, atol=1e-13)


@pytest.mark.parametrize("radius", [1, 2, 4])
def test_dimension_reduction(oracle_mod, radius):
    """A 3D field constant along one axis evolves like the 2D stencil on the
    other two axes, with that axis' coefficients folded into the centre.
    Done for z (keeps x, y) and for x (2D sees y as its x, z as its y): pins
    the axis each direction pair acts on."""
    c3 = synth.coefficients(9, 3, radius).astype(np.float64)
    g = synth.grid_uniform(21, (8, 11)).astype(np.float64)  # (ny, nx)
    # constant in z
    f3 = np.broadcast_to(g, (6, 8, 11)).copy()
    c2 = np.zeros(1 + 4 * radius)
    c2[0] = c3[0] + sum(c3[coef_index(3, "B", i)] + c3[coef_index(3, "A", i)] for i in range(1, radius + 1))
    for i in range(1, radius + 1):
        for d in "WESN":
            c2[coef_index(2, d, i)] = c3[coef_index(3, d, i)]
    out3 = oracle_mod.star_run_f64(f3, c3, radius, 3)
    out2 = oracle_mod.star_run_f64(g, c2, radius, 3)
    for zz in range(6):
        np.testing.assert_allclose(out3[zz], out2, rtol=1e-13, atol=1e-14)
    # constant in x: numpy shape (nz, ny, nx); the 2D grid is (nz, ny) -> its x is y
    h = synth.grid_uniform(22, (7, 9)).astype(np.float64)  # (nz, ny)
    f3 = np.repeat(h[:, :, None], 5, axis=2)
    c2 = np.zeros(1 + 4 * radius)
    c2[0] = c3[0] + sum(c3[coef_index(3, "W", i)] + c3[coef_index(3, "E", i)] for i in range(1, radius + 1))
    for i in range(1, radius + 1):
        for d2, d3 in (("W", "S"), ("E", "N"), ("S", "B"), ("N", "A")):
            c2[coef_index(2, d2, i)] = c3[coef_index(3, d3, i)]
    out3 = oracle_mod.star_run_f64(f3, c3, radius, 2)
    out2 = oracle_mod.star_run_f64(h, c2, radius, 2)
    for xx in range(5):
        np.testing.assert_allclose(out3[:, :, xx], out2, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("shape", [(20, 30), (9, 10, 11)])
def test_max_principle(oracle_mod, shape):
    ndim = len(shape)
    for radius in (1, 4):
        c = synth.coefficients(77, ndim, radius)
        drift = abs(float(np.sum(c.astype(np.float64))) - 1.0)
        f = synth.grid_uniform(8, shape)
        steps = 20
        out = oracle_mod.star_run_f64(f, c, radius, steps)
        lo, hi = float(f.min()), float(f.max())
        tol = 1e-12 + steps * drift
        assert out.min() >= lo * (1 - tol) - tol and out.max() <= hi * (1 + tol) + tol
        assert out.max() - out.min() < hi - lo  # diffusion shrinks the range


@pytest.mark.parametrize("shape", [(12, 15), (6, 7, 8)])
def test_mirror_symmetry(oracle_mod, shape):
    """Flipping x and swapping every W/E coefficient pair flips the result."""
    ndim = len(shape)
    radius = 3
    c = synth.coefficients(13, ndim, radius).astype(np.float64)
    cm = c.copy()
    for i in range(1, radius + 1):
        w, e = coef_index(ndim, "W", i), coef_index(ndim, "E", i)
        cm[w], cm[e] = c[e], c[w]
    f = synth.grid_uniform(14, shape).astype(np.float64)
    a = oracle_mod.star_run_f64(f, c, radius, 4)
    b = oracle_mod.star_run_f64(np.flip(f, axis=-1), cm, radius, 4)
    np.testing.assert_allclose(np.flip(b, axis=-1), a, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("shape", [(31, 29), (7, 9, 8)])
def test_step_composition_bitwise(oracle_mod, shape):
    ndim = len(shape)
    c = synth.coefficients(3, ndim, 2)
    f = synth.grid_uniform(4, shape)
    for run in (oracle_mod.star_run_f64, oracle_mod.star_run_f32):
        whole = run(f, c, 2, 7)
        part = run(run(f, c, 2, 3), c, 2, 4)
        np.testing.assert_array_equal(whole, part)
        np.testing.assert_array_equal(run(f, c, 2, 0), f.astype(whole.dtype))


@pytest.mark.parametrize("shape,radius,steps", [((64, 80), 1, 50), ((64, 70), 4, 50),
                                                ((20, 24, 28), 1, 30), ((20, 24, 28), 4, 30)])
def test_f32_form_within_rounding_bound(oracle_mod, shape, radius, steps):
    """The single-precision form stays within the a priori bound
    steps * points * 2^-24 (normwise, relative) of the FP64 definition, and
    in practice well inside 1e-5."""
    ndim = len(shape)
    c = synth.coefficients(50 + radius, ndim, radius)
    f = synth.grid_uniform(51, shape)
    ref = oracle_mod.star_run_f64(f, c, radius, steps)
    got = oracle_mod.star_run_f32(f, c, radius, steps)
    err = oracle_mod.rel_linf(got, ref)
    assert err <= steps * (1 + 2 * ndim * radius) * 2.0 ** -24
    assert err <= 1e-5
    assert err > 0  # the two forms do round differently


@pytest.mark.parametrize("shape,radius,steps", [((40, 37), 3, 5), ((11, 13, 9), 2, 4),
                                                ((3, 50), 4, 3), ((7, 2, 5), 4, 2)])
def test_sampled_cells_match_full_sweep(oracle_mod, shape, radius, steps):
    """The dependence-cone evaluation equals the full sweep bit for bit."""
    ndim = len(shape)
    c = synth.coefficients(31, ndim, radius)
    f = synth.grid_uniform(32, shape)
    full = oracle_mod.star_run_f64(f, c, radius, steps)
    rng = np.random.default_rng(0)
    dims = shape[::-1]
    cells = np.stack([rng.integers(0, n, size=40) for n in dims], axis=1)
    corners = np.array([[0] * ndim, [n - 1 for n in dims]])
    cells = np.concatenate([cells, corners])
    vals = oracle_mod.star_sample_f64(f, c, radius, steps, cells)
    want = np.array([full[tuple(p[::-1])] for p in cells])
    np.testing.assert_array_equal(vals, want)
    # the single-precision cone evaluation equals the single-precision sweep
    full32 = oracle_mod.star_run_f32(f, c, radius, steps)
    vals32 = oracle_mod.star_sample_f32(f, c, radius, steps, cells)
    np.testing.assert_array_equal(vals32, np.array([full32[tuple(p[::-1])] for p in cells]))


def test_invalid_arguments(oracle_mod):
    f = np.zeros((4, 4), dtype=np.float32)
    with pytest.raises(ValueError):
        oracle_mod.star_run_f64(f, np.zeros(4), 1, 1)  # wrong point count
    with pytest.raises(ValueError):
        oracle_mod.star_run_f64(f, np.zeros(5), 1, -1)
    with pytest.raises(ValueError):
        oracle_mod.star_run_f64(f, np.zeros(1), 0, 1)


# --- Table I, Table III, Tables IV/V and Eq. (3) --------------------------

def test_table1_flop_and_bytes(oracle_mod):
    for nd, r, flop, byte, ratio in golden("table1_stencil_characteristics.txt"):
        nd, r = int(nd), int(r)
        assert oracle_mod.flop_per_cell(nd, r) == int(flop)
        assert oracle_mod.bytes_per_cell(4) == int(byte)
        assert oracle_mod.flop_per_cell(nd, r) / oracle_mod.bytes_per_cell(4) == float(ratio)


def test_table3_derived_columns(oracle_mod):
    """GFLOP/s and GB/s are GCell/s times Table I's FLOP and bytes."""
    for row in golden("table3_fpga_results.txt"):
        nd, r = int(row[0]), int(row[1])
        gbs, gfl, gc = map(float, row[9:12])
        assert abs(oracle_mod.gflops(gc, nd, r) - gfl) <= 0.025
        assert abs(oracle_mod.gbytes_per_s(gc) - gbs) <= 0.025


def test_eq3_orientation_from_minimum_runtime(oracle_mod):
    """cells * iterations / GCell/s reproduces Sec. IV.C's minimum run times."""
    floors = {int(a): float(b) for a, b in golden("min_runtime.txt")}
    t = {2: [], 3: []}
    for row in golden("table3_fpga_results.txt"):
        nd = int(row[0])
        nx, ny, nz = int(row[6]), int(row[7]), int(row[8])
        gc = float(row[11])
        cells = nx * ny * nz
        seconds = cells * 1000 / (gc * 1e9)
        assert abs(oracle_mod.gcells_per_s(cells, 1000, seconds) - gc) < 1e-9
        t[nd].append(seconds)
    for nd, floor in floors.items():
        assert floor <= min(t[nd]) < floor + 1


def test_table3_sizes_are_compute_block_multiples():
    """Eq. (2): csize = bsize - 2 * par_time * rad divides every input side."""
    for row in golden("table3_fpga_results.txt"):
        nd, r = int(row[0]), int(row[1])
        bx, by, pt = int(row[2]), int(row[3]), int(row[5])
        nx, ny = int(row[6]), int(row[7])
        cx = bx - 2 * pt * r
        assert nx % cx == 0
        if nd == 3:
            assert ny % (by - 2 * pt * r) == 0


def test_roofline_ratios(oracle_mod):
    for dev, nd, r, gc, peak, ratio in golden("roofline_ratio.txt"):
        got = oracle_mod.roofline_ratio(oracle_mod.gbytes_per_s(float(gc)), float(peak))
        assert abs(got - float(ratio)) <= 0.005 + 1e-9, (dev, nd, r, got, ratio)
