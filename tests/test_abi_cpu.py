"""Host-side checks of the C-ABI library: it loads, exports every symbol the
header declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "stencil.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"STENCIL_API\s+[\w\s\*]*?\b(stencil_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2002_05983_amd import stencil
    if not os.path.exists(stencil.LIB_PATH):
        pytest.fail("library not built: run __graft_entry__.build()")
    return stencil.load()


def test_header_declares_the_abi():
    names = declared_functions()
    for must in ("stencil_plan", "stencil_plan_ex", "stencil_run", "stencil_run_batched",
                 "stencil_batch_create", "stencil_batch_launch", "stencil_batch_autotune",
                 "stencil_plan_query", "stencil_reduce_f64", "stencil_plan_destroy",
                 "stencil_status_string", "stencil_last_error"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2002_05983_amd import stencil
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in stencil.SIGNATURES, f"binding lacks {name}"


def test_only_the_abi_is_exported():
    import subprocess
    from paper_2002_05983_amd import stencil
    out = subprocess.run(["nm", "-D", "--defined-only", stencil.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    ours = [l.split()[-1] for l in out.splitlines() if l.split()[-1].startswith(("stencil", "_Z"))]
    leaked = [s for s in ours if "plan" in s and not s.startswith("stencil_")]
    assert not leaked, leaked


def test_status_strings_and_version(lib):
    assert lib.stencil_status_string(0) == b"ok"
    assert lib.stencil_status_string(-1) == b"invalid argument"
    assert lib.stencil_version().startswith(b"mi355x-stencil")


def _plan(lib, ndim, dims, radius, coeffs, ncoeffs=None, boundary=0, storage=0, anchor=0, tune=None):
    h = ctypes.c_void_p()
    d = (ctypes.c_int64 * max(1, len(dims)))(*dims)
    c = (ctypes.c_float * max(1, len(coeffs)))(*coeffs)
    rc = lib.stencil_plan_ex(ctypes.byref(h), ndim, d, radius, c,
                             len(coeffs) if ncoeffs is None else ncoeffs, boundary, storage, anchor,
                             tune)
    return rc, h


@pytest.mark.parametrize("case", [
    dict(ndim=1, dims=[4], radius=1, coeffs=[0.0] * 3),
    dict(ndim=4, dims=[4] * 4, radius=1, coeffs=[0.0] * 9),
    dict(ndim=2, dims=[4, 4], radius=0, coeffs=[0.0]),
    dict(ndim=2, dims=[4, 4], radius=9, coeffs=[0.0] * 37),
    dict(ndim=2, dims=[4, 4], radius=1, coeffs=[0.0] * 4),
    dict(ndim=3, dims=[4, 4, 4], radius=2, coeffs=[0.0] * 9),
    dict(ndim=2, dims=[0, 4], radius=1, coeffs=[0.0] * 5),
    dict(ndim=2, dims=[4, -3], radius=1, coeffs=[0.0] * 5),
    dict(ndim=2, dims=[4, 4], radius=1, coeffs=[0.0] * 5, boundary=2),
    dict(ndim=2, dims=[4, 4], radius=1, coeffs=[0.0] * 5, storage=7),
    dict(ndim=2, dims=[4, 4], radius=1, coeffs=[0.0] * 5, storage=1, anchor=0),
    dict(ndim=2, dims=[4, 4], radius=1, coeffs=[float("nan")] + [0.0] * 4),
    dict(ndim=3, dims=[1 << 20, 1 << 20, 1 << 20], radius=1, coeffs=[0.0] * 7),
])
def test_plan_rejects_invalid_arguments(lib, case):
    rc, h = _plan(lib, **case)
    assert rc == -1, (case, rc, lib.stencil_last_error())
    assert not h.value
    assert lib.stencil_last_error()


def test_plan_radius_limits(lib):
    """Radius 1..8 in 2D and 3D.  In 3D, K is at most 2 at radius 5, 6
    and 1 at radius 7, 8 (a larger k is invalid), and low-precision storage
    is a valid request the library does not support above radius 4.  Decided
    before any device call."""
    for ndim in (2, 3):
        rc, h = _plan(lib, ndim, [4] * ndim, 9, [0.0] * (1 + 2 * ndim * 9))
        assert rc == -1 and not h.value
    for radius, kbad in ((5, 3), (6, 3), (7, 2), (8, 2)):
        c = [0.0] * (1 + 6 * radius)
        rc, h = _plan(lib, 3, [16, 16, 16], radius, c, storage=1, anchor=3)
        assert rc == -4 and not h.value, (radius, rc)
        assert b"radius 1..4" in lib.stencil_last_error()
        rc, h = _plan(lib, 3, [16, 16, 16], radius, c, tune=b"k=%d" % kbad)
        assert rc == -1 and not h.value, (radius, rc)
    for radius, kbad in ((1, 5), (2, 4), (3, 4), (4, 3)):
        c = [0.0] * (1 + 6 * radius)
        rc, h = _plan(lib, 3, [16, 16, 16], radius, c, tune=b"k=%d" % kbad)
        assert rc == -1 and not h.value, (radius, rc)


def test_plan_null_out_pointer(lib):
    d = (ctypes.c_int64 * 2)(4, 4)
    c = (ctypes.c_float * 5)()
    assert lib.stencil_plan(None, 2, d, 1, c, 5, 0) == -1


def test_run_and_reduce_reject_null(lib):
    assert lib.stencil_run(None, None, None, 1, None) == -1
    out = (ctypes.c_double * 3)()
    assert lib.stencil_reduce_f64(None, None, 4, out, None) == -1
    assert lib.stencil_run_batched(-1, None, None, None, None, None) == -1
    assert lib.stencil_run_batched(0, None, None, None, None, None) == 0
    lib.stencil_plan_destroy(None)


def test_batch_entry_points_reject_null(lib):
    h = ctypes.c_void_p()
    assert lib.stencil_batch_create(None, 1, None, None, None, None, None) == -1
    assert lib.stencil_batch_create(ctypes.byref(h), 0, None, None, None, None, None) == -1
    assert not h.value
    assert lib.stencil_batch_create(ctypes.byref(h), 2, None, None, None, None, None) == -1
    assert b"NULL" in lib.stencil_last_error()
    plans = (ctypes.c_void_p * 1)(None)
    ptrs = (ctypes.c_void_p * 1)(None)
    steps = (ctypes.c_int64 * 1)(1)
    assert lib.stencil_batch_create(ctypes.byref(h), 1, plans, ptrs, ptrs, steps, None) == -1
    assert lib.stencil_run_batched(1, plans, ptrs, ptrs, steps, None) == -1
    assert lib.stencil_batch_launch(None, None) == -1
    assert lib.stencil_batch_autotune(None, None, 0, None) == -1
    assert lib.stencil_batch_describe(None, None, 0) == -1
    lib.stencil_batch_destroy(None)


@pytest.mark.parametrize("ndim,dims,radius,tune,ok", [
    (2, [64, 64], 1, b"k=8,ly=128", True),
    (2, [64, 64], 1, b"k=10,ly=64", True),   # up to 10 fused steps at R = 1
    (2, [64, 64], 1, b"k=11", False),
    (2, [64, 64], 4, b"k=4,ly=16", True),
    (2, [64, 64], 4, b"k=5", False),          # K*R > 16 is not built
    (2, [64, 64], 1, b"k=0", False),
    (2, [64, 64], 1, b"ly=0", False),
    (2, [64, 64], 1, b"lz=4", False),         # 3D-only key
    (2, [64, 64], 1, b"naive", True),
    (3, [64, 64, 64], 1, b"k=4,wl=32,lz=16", True),
    (3, [512, 64, 64], 2, b"k=1,vec=8,wl=64", True),
    (3, [512, 64, 64], 2, b"k=1,vec=8,wl=32", False),   # wide rows need 64 lanes
    (3, [510, 64, 64], 1, b"k=1,vec=8,wl=64", False),   # ... and 16-byte rows
    (3, [512, 64, 64], 3, b"k=1,vec=8,wl=64", False),   # ... and R <= 2
    (3, [64, 64, 64], 2, b"k=4", False),
    (3, [64, 64, 64], 3, b"k=3", True),
    (3, [64, 64, 64], 4, b"k=2", True),
    (3, [64, 64, 64], 4, b"k=3", False),
    (3, [64, 64, 64], 4, b"k=2,nw=16,wl=64", False),    # 16 rows < 2*K*R+1
    (3, [64, 64, 64], 4, b"k=1,nw=4,wl=64", False),     # 4 rows < 2*K*R+1
    (3, [64, 64, 64], 4, b"k=1,nw=5,wl=32", True),
    (3, [64, 64, 64], 1, b"wl=16", False),
    (3, [64, 64, 64], 4, b"k=1,rows=2,nbp=1,lz=32", True),
    (3, [64, 64, 64], 5, b"k=1,rows=1,nbp=0", True),
    (3, [64, 64, 64], 5, b"k=1,rows=2", True),           # two rows per wavefront above R = 4 ...
    (3, [64, 64, 64], 6, b"k=1,rows=2,nbp=1", False),    # ... without neighbour prefetch
    (3, [64, 64, 64], 4, b"k=1,rows=4,nbp=0", True),     # four rows, no neighbour prefetch
    (3, [64, 64, 64], 4, b"k=1,rows=4,nbp=1", False),
    (3, [64, 64, 64], 5, b"k=1,rows=4", False),
    (3, [63, 64, 64], 2, b"k=1,rows=2", False),          # ... on 16-byte rows
    (3, [63, 64, 64], 2, b"k=1,rows=1,nbp=1", False),
    (3, [63, 64, 64], 2, b"k=1,rows=1,nbp=0", True),
    (3, [64, 64, 64], 2, b"k=2,rows=1", False),          # single-step layout
    (3, [64, 64, 64], 2, b"k=1,rows=3", False),
    (3, [64, 64, 64], 4, b"k=1,lz=16,lpr=16", True),       # 16 lanes per row, 16-byte rows ...
    (3, [63, 64, 64], 4, b"k=1,rows=1,nbp=0,lpr=16", True),  # ... or not
    (3, [64, 64, 64], 5, b"k=1,lpr=16", False),             # radius <= 4
    (3, [64, 64, 64], 2, b"k=1,rows=2,lpr=16", False),      # one row per lane group
    (3, [64, 64, 64], 2, b"k=1,nbp=1,lpr=16", False),       # no neighbour prefetch
    (3, [64, 64, 64], 2, b"k=1,lpr=32", False),
    (3, [64, 64, 64], 2, b"k=2,lpr=16", False),             # single-step layout
    (3, [64, 64, 64], 2, b"k=1,nbp=2", False),
    (3, [64, 64, 64], 1, b"k=2,bogus=3", False),
    (3, [64, 64, 64], 1, b"k=x", False),
])
def test_tune_strings_are_validated_before_the_device(lib, ndim, dims, radius, tune, ok):
    c = [0.1] * (1 + 2 * ndim * radius)
    rc, h = _plan(lib, ndim, dims, radius, c, tune=tune)
    if ok:
        # valid: fails only because there is no device here (or succeeds on a GPU host)
        assert rc in (0, -3), (rc, lib.stencil_last_error())
        if rc == 0:
            lib.stencil_plan_destroy(h)
    else:
        assert rc == -1, (rc, lib.stencil_last_error())


def test_3d_plane_limit_is_checked_before_the_device(lib):
    # 8 x 67108864 cells x 4 B = 2^31 bytes per plane: beyond 32-bit plane offsets
    c = [0.1] * 7
    rc, h = _plan(lib, 3, [67108864, 8, 2], 1, c)
    assert rc == -4 and not h.value, (rc, lib.stencil_last_error())
    assert b"2^31" in lib.stencil_last_error()


def test_2d_row_limit_is_checked_before_the_device(lib):
    # 2^29 + 1 columns x 4 B exceed the 2^31-byte row descriptor of the 2D kernels
    c = [0.2] * 5
    rc, h = _plan(lib, 2, [(1 << 29) + 1, 2], 1, c)
    assert rc == -4 and not h.value, (rc, lib.stencil_last_error())
    assert b"2^31" in lib.stencil_last_error()


def test_coeffs_per_direction_expands_by_hand(lib):
    """One value per direction (Sec. IV.A's instance) expands to the same
    value at every distance, in the per-point order."""
    src = (ctypes.c_float * 7)(0.4, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6)
    out = (ctypes.c_float * 13)()
    assert lib.stencil_coeffs_per_direction(3, 2, src, out) == 0
    want = [0.4] + [0.1, 0.2, 0.3, 0.4, 0.5, 0.6] * 2
    assert [round(v, 6) for v in out] == [round(v, 6) for v in want]
    src2 = (ctypes.c_float * 5)(1, 2, 3, 4, 5)
    out2 = (ctypes.c_float * 13)()
    assert lib.stencil_coeffs_per_direction(2, 3, src2, out2) == 0
    assert list(out2) == [1.0] + [2.0, 3.0, 4.0, 5.0] * 3
    assert lib.stencil_coeffs_per_direction(4, 1, src, out) == -1
    assert lib.stencil_coeffs_per_direction(2, 0, src, out) == -1
    assert lib.stencil_coeffs_per_direction(2, 1, None, out) == -1


def _plan_sym(lib, ndim, dims, radius, coeffs, boundary=0, tune=None):
    h = ctypes.c_void_p()
    d = (ctypes.c_int64 * ndim)(*dims)
    c = (ctypes.c_float * max(1, len(coeffs)))(*coeffs)
    rc = lib.stencil_plan_symmetric(ctypes.byref(h), ndim, d, radius, c, len(coeffs), boundary,
                                    tune)
    return rc, h


@pytest.mark.parametrize("ndim,radius,ncoef,boundary,tune,want", [
    (2, 2, 5, 0, None, (0, -3)),
    (2, 2, 9, 0, None, (-1,)),        # per-point count is not the shared count
    (3, 3, 10, 0, None, (0, -3)),
    (3, 5, 16, 0, None, (-4,)),       # built for radius 1..4
    (2, 2, 5, 1, None, (-4,)),        # clamp boundary only
    (2, 2, 5, 7, None, (-1,)),
    (2, 2, 5, 0, b"k=4,ly=64", (0, -3)),
    (2, 2, 5, 0, b"k=5", (-1,)),      # up to 4 fused steps
    (3, 2, 7, 0, b"k=2", (-1,)),      # 3D runs the single-step row layout
    (3, 2, 7, 0, b"k=1,wl=32,nw=16", (-1,)),
    (3, 2, 7, 0, b"k=1,rows=1,nbp=1,lz=64", (0, -3)),
    (3, 2, 7, 0, b"k=1,rows=2", (-1,)),
    (3, 2, 7, 0, b"k=1,rows=1,lpr=16", (-1,)),  # 16 lanes per row: per-point coefficients
])
def test_symmetric_plan_validation(lib, ndim, radius, ncoef, boundary, tune, want):
    rc, h = _plan_sym(lib, ndim, [64] * ndim, radius, [0.1] * ncoef, boundary, tune)
    assert rc in want, (rc, lib.stencil_last_error())
    if rc == 0:
        lib.stencil_plan_destroy(h)


def test_padded_boundary_validation(lib):
    c = [0.1] * 13
    rc, h = _plan(lib, 3, [16, 16, 16], 2, c, boundary=1)
    assert rc in (0, -3), lib.stencil_last_error()
    if rc == 0:
        lib.stencil_plan_destroy(h)
    rc, h = _plan(lib, 3, [16, 16, 16], 2, c, boundary=1, storage=1, anchor=4)
    assert rc == -4 and b"padded" in lib.stencil_last_error()
    rc, h = _plan(lib, 2, [16, 16], 2, [0.1] * 9, boundary=2)
    assert rc == -1
