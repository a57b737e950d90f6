"""Full-size parity in the launch configurations the benchmark times.

The 16384^2 2D grid at R = 1..8, the 512^3 3D grid at R = 1..8 and the
768^3 grid at R = 4 (the workloads bench.py measures, with its seeds), each
plan autotuned as bench.py does:
  * run for three passes plus a tail pass and checked on sampled cells --
    corners, face centres and random interior cells -- bitwise against the
    oracle's single-precision cone evaluation and within the FP32 tolerance
    against its FP64 one;
  * at R = 1..4, run for the same short count and compared with the
    oracle's single-precision sweep of the whole grid, every cell;
  * run for the full step counts of the workloads (1000 steps at 16384^2
    and 768^3, 200 at 512^3) and compared on stored cells with the FP64
    oracle's values (tests/golden/fp64_*.txt, written by
    tests/golden/make_fullsize_reference.py): normwise relative L-infinity
    <= 1e-5 over the stored cells, normalised by the stored max |f| of the
    whole FP64 grid, and the conservation sum within 1e-5 of the FP64 sum.
Plus the widest 3D plane the kernels accept (nx*ny*4 just under 2^31 bytes).
"""
import os

import numpy as np
import pytest

from conftest import ROOT
from paper_2002_05983_amd import synth

pytestmark = pytest.mark.gpu

TOL_F64 = 1e-5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


@pytest.fixture(scope="module")
def st():
    from paper_2002_05983_amd import stencil
    stencil.load()
    return stencil


def sample_cells(shape, n=24, seed=0):
    """(x, y[, z]) cells: every corner, every face centre, n random cells."""
    dims = shape[::-1]
    nd = len(dims)
    cells = []
    for m in range(1 << nd):
        cells.append([(dims[a] - 1) if (m >> a) & 1 else 0 for a in range(nd)])
    for a in range(nd):
        for side in (0, dims[a] - 1):
            c = [d // 2 for d in dims]
            c[a] = side
            cells.append(c)
    rng = np.random.default_rng(seed)
    cells += np.stack([rng.integers(0, d, n) for d in dims], axis=1).tolist()
    return np.array(cells, dtype=np.int64)


def check_sampled(torch, st, oracle_mod, f, c, radius, tune_first=True, what=""):
    x = torch.from_numpy(f).cuda()
    y = torch.empty_like(x)
    plan = st.Plan(f.shape, radius, c)
    if tune_first:
        plan.autotune(x, y)
    K = plan.query()["K"]
    steps = 3 * K + 1 if K > 1 else 4
    plan.run(x, y, steps)
    torch.cuda.synchronize()
    cells = sample_cells(f.shape)
    idx = tuple(cells[:, a] for a in range(cells.shape[1]))[::-1]
    got = y.cpu().numpy()[idx]
    want32 = oracle_mod.star_sample_f32(f, c, radius, steps, cells)
    desc = plan.describe()
    assert np.array_equal(got, want32), (what, desc, np.argwhere(got != want32)[:5].tolist())
    want64 = oracle_mod.star_sample_f64(f, c, radius, steps, cells)
    err = np.max(np.abs(got - want64)) / np.max(np.abs(want64))
    assert err <= TOL_F64, (what, desc, err)
    plan.close()
    return desc


@pytest.fixture(scope="module")
def grid2d():
    return synth.grid_uniform(1, (16384, 16384))


@pytest.mark.parametrize("radius", [1, 2, 3, 4, 5, 6, 7, 8])
def test_2d_16384sq_bench_configuration(torch, st, oracle_mod, grid2d, radius):
    c = synth.coefficients(1000 + radius, 2, radius)
    check_sampled(torch, st, oracle_mod, grid2d, c, radius, what=f"2D R{radius}")


@pytest.fixture(scope="module")
def grid3d():
    return synth.grid_uniform(2, (512, 512, 512))


@pytest.mark.parametrize("radius", [1, 2, 3, 4, 5, 6, 7, 8])
def test_3d_512cube_bench_configuration(torch, st, oracle_mod, grid3d, radius):
    c = synth.coefficients(2000 + radius, 3, radius)
    check_sampled(torch, st, oracle_mod, grid3d, c, radius, what=f"3D R{radius}")


def test_3d_768cube_r4_bench_configuration(torch, st, oracle_mod):
    f = synth.sinusoid_grid(4, 768)
    c = synth.coefficients(3004, 3, 4)
    check_sampled(torch, st, oracle_mod, f, c, 4, what="768^3 R4")


def test_2d_grid_beyond_2_31_cells(torch, st, oracle_mod):
    """33000 x 65536 = 2.16e9 cells (> 2^31; 8.65 GB per grid): row offsets
    and the store descriptors must not wrap in 32 bits."""
    shape = (33000, 65536)
    f = synth.grid_uniform(9, shape)
    c = synth.coefficients(10, 2, 3)
    check_sampled(torch, st, oracle_mod, f, c, 3, tune_first=False, what="2D 2.16e9 cells")


def test_widest_3d_plane(torch, st, oracle_mod):
    """nx*ny*4 = 2^31 - 128 bytes per plane: the largest plane the 3D
    kernels address with 32-bit offsets."""
    shape = (2, 8, 67108860)
    f = synth.grid_uniform(7, shape)
    c = synth.coefficients(8, 3, 1)
    check_sampled(torch, st, oracle_mod, f, c, 1, tune_first=False, what="widest plane")
    with pytest.raises(st.StencilError):  # one more row of 4 cells crosses 2^31 bytes
        st.Plan((2, 8, 67108864), 1, c)


# --- every cell, short runs ---------------------------------------------------

def check_every_cell(torch, st, oracle_mod, f, c, radius, what):
    x = torch.from_numpy(f).cuda()
    y = torch.empty_like(x)
    plan = st.Plan(f.shape, radius, c)
    plan.autotune(x, y)
    K = plan.query()["K"]
    steps = 3 * K + 1
    plan.run(x, y, steps)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    desc = plan.describe()
    plan.close()
    del x, y
    want = oracle_mod.star_run_f32(f, c, radius, steps)
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{what} [{desc}] {steps} steps: {len(bad)} cells differ, "
                             f"first {bad[:5].tolist()}")


@pytest.mark.parametrize("radius", [1, 2, 3, 4])
def test_2d_16384sq_every_cell(torch, st, oracle_mod, grid2d, radius):
    c = synth.coefficients(1000 + radius, 2, radius)
    check_every_cell(torch, st, oracle_mod, grid2d, c, radius, f"2D R{radius}")


@pytest.mark.parametrize("radius", [1, 2, 3, 4])
def test_3d_512cube_every_cell(torch, st, oracle_mod, grid3d, radius):
    c = synth.coefficients(2000 + radius, 3, radius)
    check_every_cell(torch, st, oracle_mod, grid3d, c, radius, f"3D R{radius}")


# --- FP64 at the workloads' full step counts ----------------------------------

GOLDEN_FP64 = ["2d16k_r1", "2d16k_r2", "2d16k_r3", "2d16k_r4",
               "3d512_r1", "3d512_r2", "3d512_r3", "3d512_r4", "3d768sin_r4"]


def read_fp64_reference(name):
    """Header fields and (cells, values) of tests/golden/fp64_<name>.txt."""
    meta, cells, vals = {}, [], []
    with open(os.path.join(ROOT, "tests", "golden", f"fp64_{name}.txt")) as fh:
        for line in fh:
            if line.startswith("#"):
                parts = line[1:].split()
                if len(parts) >= 2 and parts[0] in ("dims", "radius", "steps", "grid",
                                                    "coef_seed", "maxabs", "sum"):
                    meta[parts[0]] = parts[1:]
                continue
            t = line.split()
            cells.append([int(v) for v in t[:-1]])
            vals.append(float(t[-1]))
    return meta, np.array(cells, dtype=np.int64), np.array(vals)


def fp64_workload(meta):
    dims = [int(v) for v in meta["dims"]]
    kind, seed = meta["grid"][0], int(meta["grid"][1])
    shape = tuple(dims[::-1])
    f = synth.grid_uniform(seed, shape) if kind == "uniform" else synth.sinusoid_grid(seed, dims[0])
    radius = int(meta["radius"][0])
    c = synth.coefficients(int(meta["coef_seed"][0]), len(dims), radius)
    return f, c, radius, int(meta["steps"][0])


@pytest.mark.parametrize("name", GOLDEN_FP64)
def test_fp64_parity_at_full_step_count(torch, st, name):
    """FP32 within 1e-5 (normwise relative L-infinity) of FP64 after the
    workload's full step count, in the autotuned configuration."""
    meta, cells, want = read_fp64_reference(name)
    f, c, radius, steps = fp64_workload(meta)
    x = torch.from_numpy(f).cuda()
    del f
    y = torch.empty_like(x)
    plan = st.Plan(tuple(x.shape), radius, c)
    plan.autotune(x, y)
    plan.run(x, y, steps)
    torch.cuda.synchronize()
    idx = tuple(torch.from_numpy(cells[:, a]).cuda() for a in range(cells.shape[1] - 1, -1, -1))
    got = y[idx].double().cpu().numpy()
    maxabs = float(meta["maxabs"][0])
    err = float(np.max(np.abs(got - want))) / maxabs
    _, _, total = st.reduce_f64(y, None)
    want_sum = float(meta["sum"][0])
    desc = plan.describe()
    plan.close()
    print(f"{name}: rel-Linf {err:.3e} over {len(cells)} cells, sum rel diff "
          f"{abs(total - want_sum) / abs(want_sum):.3e} [{desc}]", flush=True)
    assert err <= TOL_F64, (name, desc, err)
    assert abs(total - want_sum) <= TOL_F64 * abs(want_sum), (name, desc, total, want_sum)
