"""Full-size parity in the launch configurations the benchmark times.

The 16384^2 2D grid at R = 1..8, the 512^3 3D grid at R = 1..8 and the
768^3 grid at R = 4 (the workloads bench.py measures, with its seeds), each
plan autotuned as bench.py does, run for three passes plus a tail pass, and
checked on sampled cells -- corners, face centres and random interior
cells -- bitwise against the oracle's single-precision cone evaluation and
within the FP32 tolerance against its FP64 one.  Plus the widest 3D plane
the kernels accept (nx*ny*4 just under 2^31 bytes).
"""
import numpy as np
import pytest

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
