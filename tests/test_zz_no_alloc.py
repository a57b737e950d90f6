"""stencil_run_noalloc against stencil_run, through the C ABI.

The allocation-free entry point runs the same kernels with the library's
static partner grid: its result must equal stencil_run's bit for bit (and
so the oracle's single-precision form), call after call on one device --
here a larger grid, then a smaller one that reuses the same static array.
"""
import ctypes

import numpy as np
import pytest

from paper_2002_05983_amd import synth

pytestmark = pytest.mark.gpu


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


def run_both(torch, st, shape, radius, steps, tune=None):
    c = synth.coefficients(4100 + radius, len(shape), radius)
    f = synth.grid_uniform(4200 + radius, shape)
    plan = st.Plan(shape, radius, c, tune=tune)
    x = torch.from_numpy(f).cuda()
    y_run = torch.full_like(x, float("nan"))
    y_static = torch.full_like(x, float("nan"))
    stream = torch.cuda.current_stream()
    lib = st.load()
    rc = lib.stencil_run(plan.handle, x.data_ptr(), y_run.data_ptr(), steps, int(stream.cuda_stream))
    assert rc == 0, lib.stencil_last_error()
    rc = lib.stencil_run_noalloc(plan.handle, x.data_ptr(), y_static.data_ptr(), steps,
                                 int(stream.cuda_stream))
    assert rc == 0, lib.stencil_last_error()
    torch.cuda.synchronize()
    a, b = y_run.cpu().numpy(), y_static.cpu().numpy()
    assert np.array_equal(x.cpu().numpy(), f)  # in is never written
    desc = plan.describe()
    plan.close()
    return a, b, f, c, desc


def test_noalloc_equals_run_on_two_calls(torch, st, oracle_mod):
    # first a 3D grid of 1.6e6 cells with K = 2 passes and a tail pass ...
    a, b, f, c, desc = run_both(torch, st, (48, 160, 210), 2, 7, tune="k=2,wl=32,nw=16,lz=32")
    assert np.array_equal(a, b), desc
    assert np.array_equal(b, oracle_mod.star_run_f32(f, c, 2, 7)), desc
    # ... then a smaller 2D grid through the same static array
    a, b, f, c, desc = run_both(torch, st, (300, 517), 3, 9, tune="k=4,ly=64")
    assert np.array_equal(a, b), desc
    assert np.array_equal(b, oracle_mod.star_run_f32(f, c, 3, 9)), desc
    # and one step (a single pass: the static array is not touched) and zero steps
    for steps in (1, 0):
        a, b, f, c, desc = run_both(torch, st, (33, 70), 1, steps)
        assert np.array_equal(a, b), desc


def test_noalloc_rejects_what_it_cannot_run(torch, st):
    lib = st.load()
    # a grid above the static array's capacity (STENCIL_NOALLOC_MAX_CELLS = 2^24)
    shape = (4097, 4096)
    assert shape[0] * shape[1] > 1 << 24
    plan = st.Plan(shape, 1, synth.coefficients(1, 2, 1))
    x = torch.zeros(shape, device="cuda")
    y = torch.empty_like(x)
    rc = lib.stencil_run_noalloc(plan.handle, x.data_ptr(), y.data_ptr(), 3, None)
    assert rc == -4 and b"STENCIL_NOALLOC_MAX_CELLS" in lib.stencil_last_error()
    plan.close()
    # low-precision storage keeps plan-owned buffers
    shape = (16, 16, 16)
    plan = st.Plan(shape, 1, synth.coefficients(2, 3, 1), storage="f16", anchor_m=10)
    x = torch.zeros(shape, device="cuda")
    y = torch.empty_like(x)
    rc = lib.stencil_run_noalloc(plan.handle, x.data_ptr(), y.data_ptr(), 3, None)
    assert rc == -4
    plan.close()
