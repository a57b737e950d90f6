"""GPU parity: the HIP path against the CPU oracle, through the C ABI.

Bar: bitwise equality with the oracle's single-precision form (same
operation order), and normwise relative L-infinity <= 1e-5 against the FP64
definition (the library's stated FP32 tolerance).  Sizes span several tiles
and segments with ragged tails; edge cases cover sides of 1, sides smaller
than the radius, and step counts that leave a tail pass.
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


def gpu_run(torch, st, f, radius, coeffs, steps, tune=None):
    plan = st.Plan(f.shape, radius, coeffs, tune=tune)
    x = torch.from_numpy(f).cuda()
    y = torch.empty_like(x)
    plan.run(x, y, steps)
    torch.cuda.synchronize()
    out = y.cpu().numpy()
    # the input is never written
    assert np.array_equal(x.cpu().numpy(), f)
    desc = plan.describe()
    plan.close()
    return out, desc


def assert_bitwise(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{what}: {len(bad)} cells differ, first at {bad[:5].tolist()}, "
                             f"got {got[tuple(bad[0])]!r} want {want[tuple(bad[0])]!r}")


NAIVE_CASES = [((1, 1), 1), ((3, 2), 4), ((17, 33), 2), ((64, 100), 3), ((5, 200), 4),
               ((2, 3), 8), ((40, 70), 5), ((19, 260), 6), ((33, 17), 7),
               ((1, 1, 1), 2), ((4, 5, 6), 3), ((9, 17, 33), 1), ((3, 40, 7), 4)]


@pytest.mark.parametrize("shape,radius", NAIVE_CASES)
def test_naive_matches_oracle_bitwise(torch, st, oracle_mod, shape, radius):
    c = synth.coefficients(200 + radius, len(shape), radius)
    f = synth.grid_uniform(300 + radius, shape)
    for steps in (0, 1, 5):
        got, desc = gpu_run(torch, st, f, radius, c, steps, tune="naive")
        assert "variant=naive" in desc
        assert_bitwise(got, oracle_mod.star_run_f32(f, c, radius, steps), f"naive {shape} r{radius}")


# (ny, nx) shapes: aligned and ragged x, several strips, several segments.
S2D_SHAPES = [(1, 1), (1, 7), (6, 1), (3, 3), (2, 5), (37, 513), (97, 1000), (130, 1024),
              (64, 2048), (300, 260), (11, 4096)]


@pytest.mark.parametrize("radius", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("shape", S2D_SHAPES)
def test_s2d_matches_oracle_bitwise(torch, st, oracle_mod, radius, shape):
    c = synth.coefficients(400 + radius, 2, radius)
    f = synth.grid_uniform(500 + radius, shape)
    cache = {}
    for K in (1, 2, 3, 4, 5, 8, 10):
        if K * radius > 16:
            continue
        for ly in (7, 32):
            steps = 2 * K + 1  # two full passes and a tail pass
            if steps not in cache:
                cache[steps] = oracle_mod.star_run_f32(f, c, radius, steps)
            got, desc = gpu_run(torch, st, f, radius, c, steps, tune=f"k={K},ly={ly}")
            assert "variant=s2d" in desc, desc
            assert_bitwise(got, cache[steps], f"s2d {shape} r{radius} k{K} ly{ly}")


@pytest.mark.parametrize("radius", [1, 2, 3, 4, 5, 6, 7, 8])
def test_s2d_default_config_vs_fp64(torch, st, oracle_mod, radius):
    """Default (autoselected) configuration, 40 steps, against FP64."""
    shape = (257, 1531)
    c = synth.coefficients(600 + radius, 2, radius)
    f = synth.grid_uniform(601, shape)
    got, _ = gpu_run(torch, st, f, radius, c, 40)
    assert_bitwise(got, oracle_mod.star_run_f32(f, c, radius, 40), "s2d default")
    assert oracle_mod.rel_linf(got, oracle_mod.star_run_f64(f, c, radius, 40)) <= TOL_F64


# (nz, ny, nx) shapes: one 256- or 512-column strip, several strips, ragged x
# (unaligned), small sides, several y-tiles and z-segments.
S3D_SHAPES = [(1, 1, 1), (3, 2, 5), (4, 5, 6), (9, 17, 33), (20, 37, 300), (13, 40, 513),
              (7, 33, 600), (30, 50, 64), (6, 3, 257)]
MAX_K3D = {1: 4, 2: 3, 3: 3, 4: 2}


def s3d_tiles(K, radius):
    """(nw, lz, wl) tile shapes with at least one output row: 16- and
    32-row tiles, and the smallest tiles of each row width."""
    out = []
    for nw, lz, wl in ((16, 5, 64), (2 * K * radius + 1, 32, 64), (16, 7, 32),
                       (K * radius + 1, 3, 32)):
        if nw <= 16 and nw * (64 // wl) > 2 * K * radius:
            out.append((nw, lz, wl))
    return out


@pytest.mark.parametrize("radius", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", S3D_SHAPES)
def test_s3d_matches_oracle_bitwise(torch, st, oracle_mod, radius, shape):
    c = synth.coefficients(700 + radius, 3, radius)
    f = synth.grid_uniform(800 + radius, shape)
    cache = {}
    for K in range(1, MAX_K3D[radius] + 1):
        for nw, lz, wl in s3d_tiles(K, radius):
            steps = 2 * K + 1
            if steps not in cache:
                cache[steps] = oracle_mod.star_run_f32(f, c, radius, steps)
            got, desc = gpu_run(torch, st, f, radius, c, steps,
                                tune=f"k={K},nw={nw},lz={lz},wl={wl}")
            assert "variant=s3d" in desc, desc
            assert_bitwise(got, cache[steps], f"s3d {shape} r{radius} [{desc}]")
        if K == 1:  # two planes per barrier; odd and even plane counts per segment
            for nw, lz, wl in ((16, 5, 64), (16, 7, 32), (radius + 1, 4, 32), (16, 64, 32)):
                got, desc = gpu_run(torch, st, f, radius, c, 3,
                                    tune=f"k=1,nw={nw},lz={lz},wl={wl},pair=1")
                assert "pair=1" in desc, desc
                assert_bitwise(got, cache[3], f"s3d pair {shape} r{radius} [{desc}]")
        if K == 1 and shape[2] % 4 == 0 and 256 < shape[2] <= 512 and radius <= 2:
            got, desc = gpu_run(torch, st, f, radius, c, 3, tune="k=1,vec=8,wl=64,lz=7")
            assert "vec=8" in desc
            assert_bitwise(got, oracle_mod.star_run_f32(f, c, radius, 3), f"s3d vec8 {shape} r{radius}")


# (nz, ny, nx): one strip, several strips, ragged strips, nx not a
# multiple of 4, sides below the radius, row counts not a multiple of 2.
S3R_SHAPES = [(1, 1, 1), (3, 2, 5), (9, 17, 33), (20, 37, 300), (7, 33, 600), (13, 40, 513),
              (6, 3, 257), (11, 9, 512), (5, 6, 260), (4, 7, 768)]


@pytest.mark.parametrize("radius", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("shape", S3R_SHAPES)
def test_s3d_rows_layout_matches_oracle_bitwise(torch, st, oracle_mod, radius, shape):
    """The LDS-free single-step layout: one, two and four rows per
    wavefront (two above radius 4, four up to it), with and without
    prefetched neighbour rows, 16 lanes per row up to radius 4, segments
    shorter and longer than the grid, several passes."""
    c = synth.coefficients(720 + radius, 3, radius)
    f = synth.grid_uniform(820 + radius, shape)
    want = oracle_mod.star_run_f32(f, c, radius, 3)
    aligned = shape[2] % 4 == 0
    for rows in (1, 2, 4):
        for nbp in (0, 1):
            if rows == 4 and (nbp or radius > 4):
                continue
            if rows == 2 and radius > 4 and nbp:
                continue
            if (rows > 1 or nbp) and not aligned:
                continue
            for lz in (1, 4, 64):
                tune = f"k=1,rows={rows},nbp={nbp},lz={lz}"
                got, desc = gpu_run(torch, st, f, radius, c, 3, tune=tune)
                assert "layout=rows" in desc, desc
                assert_bitwise(got, want, f"s3d rows {shape} r{radius} [{desc}]")
    if radius <= 4:
        # 16 lanes per row: four rows of a 64-column strip per wavefront
        for lz in (1, 4, 64):
            got, desc = gpu_run(torch, st, f, radius, c, 3, tune=f"k=1,rows=1,nbp=0,lz={lz},lpr=16")
            assert "lpr=16" in desc, desc
            assert_bitwise(got, want, f"s3d rows lpr=16 {shape} r{radius} [{desc}]")


@pytest.mark.parametrize("radius", [2, 4])
def test_autotune_times_narrow_rows_only_on_narrow_grids(torch, st, oracle_mod, radius, monkeypatch):
    """Grids at most 128 cells wide are also timed with four 16-lane rows
    per wavefront; whatever the autotuner keeps is bitwise exact, and wider
    grids do not time that form."""
    monkeypatch.delenv("STENCIL_TUNE_CACHE", raising=False)
    monkeypatch.delenv("STENCIL_TUNE_TOP", raising=False)
    c = synth.coefficients(990 + radius, 3, radius)
    for shape, narrow in (((40, 33, 61), True), ((24, 20, 300), False)):
        f = synth.grid_uniform(991, shape)
        x = torch.from_numpy(f).cuda()
        y = torch.empty_like(x)
        plan = st.Plan(shape, radius, c)
        timed = [cfg for cfg, _ in plan.autotune(x, y)]
        assert any("lpr=16" in cfg for cfg in timed) == narrow, timed
        plan.run(x, y, 3)
        torch.cuda.synchronize()
        assert_bitwise(y.cpu().numpy(), oracle_mod.star_run_f32(f, c, radius, 3),
                       f"autotuned {shape} r{radius} [{plan.describe()}]")
        plan.close()


@pytest.mark.parametrize("radius", [1, 2, 3, 4])
def test_s3d_default_config_vs_fp64(torch, st, oracle_mod, radius):
    shape = (40, 45, 130)
    c = synth.coefficients(900 + radius, 3, radius)
    f = synth.grid_uniform(901, shape)
    got, _ = gpu_run(torch, st, f, radius, c, 12)
    assert_bitwise(got, oracle_mod.star_run_f32(f, c, radius, 12), "s3d default")
    assert oracle_mod.rel_linf(got, oracle_mod.star_run_f64(f, c, radius, 12)) <= TOL_F64


S3D_HIGH_SHAPES = [(1, 1, 1), (3, 4, 10), (9, 17, 33), (20, 37, 300), (6, 3, 257)]


@pytest.mark.parametrize("radius", [5, 6, 7, 8])
@pytest.mark.parametrize("shape", S3D_HIGH_SHAPES)
def test_3d_high_radius_matches_oracle_bitwise(torch, st, oracle_mod, radius, shape):
    """3D radius 5..8, sides below and above R: the default configuration,
    the single-step kernel and streaming tiles of 32 rows (two per
    wavefront) and 16 rows."""
    c = synth.coefficients(800 + radius, 3, radius)
    f = synth.grid_uniform(900 + radius, shape)
    want = {s: oracle_mod.star_run_f32(f, c, radius, s) for s in (1, 4, 5)}
    tunes = [None, "naive", "k=1,wl=32,nw=16,lz=7", "k=1,wl=32,nw=12,lz=64",
             "k=1,wl=32,nw=16,lz=9,pair=1"]
    if radius < 8:
        tunes.append("k=1,wl=64,nw=16,lz=5")  # 16 rows hold 2R halo rows up to R = 7
    if radius <= 6:  # two fused steps: 32-row tiles keep 32 - 4R > 0 output rows
        tunes += ["k=2,wl=32,nw=16,lz=6", "k=2,wl=32,nw=16,lz=64"]
    got4 = None
    for tune in tunes:
        for steps in ((1, 4, 5) if tune and tune.startswith("k=2") else (1, 4)):
            got, desc = gpu_run(torch, st, f, radius, c, steps, tune=tune)
            assert_bitwise(got, want[steps], f"3D {shape} r{radius} {desc}")
            if steps == 4:
                got4 = got
    assert oracle_mod.rel_linf(got4, oracle_mod.star_run_f64(f, c, radius, 4)) <= TOL_F64


def test_3d_high_radius_autotune(torch, st, oracle_mod):
    shape = (24, 40, 72)
    f = synth.grid_uniform(950, shape)
    c = synth.coefficients(951, 3, 6)
    plan = st.Plan(shape, 6, c)
    x = torch.from_numpy(f).cuda()
    y = torch.empty_like(x)
    rows = plan.autotune(x, y)
    cfgs = [cfg for cfg, _ in rows]
    assert "naive" in cfgs and any(cfg.startswith("k=1,wl=") for cfg in cfgs)
    assert any(cfg.startswith("k=2,") for cfg in cfgs)  # two fused steps up to radius 6
    assert all("k=3" not in cfg for cfg in cfgs)
    plan.run(x, y, 3)
    torch.cuda.synchronize()
    assert_bitwise(y.cpu().numpy(), oracle_mod.star_run_f32(f, c, 6, 3), "3D r6 tuned")
    with pytest.raises(ValueError):  # EINVAL: at most two fused steps at radius 5, 6
        st.Plan(shape, 6, c, tune="k=3")
    plan.close()


def test_config1_2d_r1_1024_10_steps(torch, st, oracle_mod):
    """2D radius 1 on 1024x1024, U[0,1) values, seeded coefficients, 10 steps."""
    c = synth.coefficients(101, 2, 1)
    f = synth.grid_uniform(1, (1024, 1024))
    got, _ = gpu_run(torch, st, f, 1, c, 10)
    assert_bitwise(got, oracle_mod.star_run_f32(f, c, 1, 10), "1024^2 r1")
    err = oracle_mod.rel_linf(got, oracle_mod.star_run_f64(f, c, 1, 10))
    assert err <= TOL_F64, err


def test_step_composition_and_zero_steps(torch, st):
    c = synth.coefficients(7, 2, 3)
    f = synth.grid_uniform(8, (200, 300))
    plan = st.Plan(f.shape, 3, c)
    x = torch.from_numpy(f).cuda()
    a, b, z = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
    plan.run(x, a, 11)
    plan.run(x, b, 4)
    plan.run(b.clone(), b, 7)
    plan.run(x, z, 0)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(z, x)


def test_run_rejects_overlap_and_bad_steps(torch, st):
    c = synth.coefficients(7, 2, 1)
    plan = st.Plan((16, 16), 1, c)
    x = torch.zeros(16, 16, device="cuda")
    with pytest.raises(ValueError):
        plan.run(x, x, 1)
    with pytest.raises(ValueError):
        plan.run(x, torch.empty_like(x), -1)
    with pytest.raises(ValueError):
        st.Plan((16, 16), 1, c, tune="k=11")
    with pytest.raises(ValueError):
        st.Plan((16, 16), 1, c, tune="bogus=1")


@pytest.mark.parametrize("n", [1, 1000, 1 << 20, 3 * (1 << 20) + 17])
def test_reduce_f64(torch, st, n):
    x = torch.from_numpy(synth.uniform01_f32(5, n)).cuda()
    ref = torch.from_numpy(synth.uniform01_f32(6, n).astype(np.float64) * 0.5).cuda()
    md, mr, sm = st.reduce_f64(x, ref)
    xn, rn = x.cpu().numpy().astype(np.float64), ref.cpu().numpy()
    assert md == np.max(np.abs(xn - rn))
    assert mr == np.max(np.abs(rn))
    assert abs(sm - np.sum(xn)) <= 1e-12 * n
    md2, mr2, sm2 = st.reduce_f64(x, None)
    assert (md2, mr2) == (0.0, 0.0) and sm2 == sm


def test_reduce_f64_propagates_nan_and_inf(torch, st):
    """A NaN or an infinite cell is reported, as numpy's max reports it."""
    n = 300_001
    base = synth.uniform01_f32(15, n)
    ref = torch.from_numpy(synth.uniform01_f32(16, n).astype(np.float64)).cuda()
    for where, val in ((7, np.nan), (n - 1, np.inf), (123_456, -np.inf)):
        xh = base.copy()
        xh[where] = val
        md, mr, sm = st.reduce_f64(torch.from_numpy(xh).cuda(), ref)
        want = np.max(np.abs(xh.astype(np.float64) - ref.cpu().numpy()))
        assert (np.isnan(md) and np.isnan(want)) or md == want, (where, val, md, want)
        assert mr == np.max(np.abs(ref.cpu().numpy()))
        assert (np.isnan(sm) and np.isnan(np.sum(xh.astype(np.float64)))) or \
            sm == np.sum(xh.astype(np.float64)) or abs(sm) == np.inf
    # a NaN in the reference shows in both maxima
    rh = ref.cpu().numpy().copy()
    rh[99] = np.nan
    md, mr, _ = st.reduce_f64(torch.from_numpy(base).cuda(), torch.from_numpy(rh).cuda())
    assert np.isnan(md) and np.isnan(mr)


@pytest.mark.parametrize("shape,radius", [((300, 700), 2), ((30, 40, 300), 1), ((20, 24, 90), 4)])
def test_autotune_keeps_bitwise_result_and_caches(torch, st, oracle_mod, shape, radius, tmp_path,
                                                  monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("STENCIL_TUNE_CACHE", str(cache))
    c = synth.coefficients(950 + radius, len(shape), radius)
    f = synth.grid_uniform(951, shape)
    x = torch.from_numpy(f).cuda()
    y = torch.empty_like(x)
    plan = st.Plan(shape, radius, c)
    table = plan.autotune(x, y)
    assert len(table) >= 2 and table[0][1] >= table[-1][1] > 0
    assert "by=autotune" in plan.describe()
    plan.run(x, y, 7)
    torch.cuda.synchronize()
    assert_bitwise(y.cpu().numpy(), oracle_mod.star_run_f32(f, c, radius, 7), "autotuned")
    # a new plan of the same problem reads the cached choice
    again = st.Plan(shape, radius, c)
    assert "by=cache" in again.describe()
    assert again.query()["K"] == plan.query()["K"]
    assert table[0][0] in cache.read_text()
    # a plan of another shape in the same size class (ceil(log2 side) per
    # axis) falls back to the class's entry, and still computes exactly
    sib_shape = tuple(n - max(1, n // 40) for n in shape)
    sib = st.Plan(sib_shape, radius, c)
    assert "by=cache" in sib.describe() and sib.query()["K"] == plan.query()["K"]
    fs = synth.grid_uniform(952, sib_shape)
    xs = torch.from_numpy(fs).cuda()
    ys = torch.empty_like(xs)
    sib.run(xs, ys, 5)
    torch.cuda.synchronize()
    assert_bitwise(ys.cpu().numpy(), oracle_mod.star_run_f32(fs, c, radius, 5), "class-cached")


# precision form: bitwise against the CPU model of the same algorithm
LOWP_SHAPES = [(70, 68, 136), (9, 70, 72), (66, 5, 300)]


@pytest.mark.parametrize("radius", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", LOWP_SHAPES)
def test_precision_form_matches_model_bitwise(torch, st, radius, shape):
    from oracle import precision
    c = synth.coefficients(1100 + radius, 3, radius)
    f = synth.sinusoid_grid(1200 + radius, max(shape), modes=4)[:shape[0], :shape[1], :shape[2]].copy()
    x = torch.from_numpy(f).cuda()
    y = torch.empty_like(x)
    for storage, codec in (("f16", precision.F16), ("bf16", precision.BF16)):
        for m, steps, tune in ((3, 7, "wl=64"), (7, 7, "wl=32,nw=12"), (1, 2, None)):
            plan = st.Plan(shape, radius, c, storage=storage, anchor_m=m, tune=tune)
            plan.run(x, y, steps)
            torch.cuda.synchronize()
            want = precision.run(f, c, radius, steps, m, codec)
            assert_bitwise(y.cpu().numpy(), want, f"{storage} m{m} {shape} r{radius} [{plan.describe()}]")
            plan.close()


@pytest.mark.parametrize("radius", [1, 2, 3, 4])
@pytest.mark.parametrize("shape", LOWP_SHAPES)
def test_scaled_state_form_matches_model_bitwise(torch, st, radius, shape):
    from oracle import precision
    c = synth.coefficients(1400 + radius, 3, radius)
    f = synth.sinusoid_grid(1500 + radius, max(shape), modes=4)[:shape[0], :shape[1], :shape[2]].copy()
    x = torch.from_numpy(f).cuda()
    y = torch.empty_like(x)
    for storage, codec in (("f16-scaled", precision.F16), ("bf16-scaled", precision.BF16)):
        for m, steps, tune in ((3, 7, "wl=64"), (7, 7, "wl=32,nw=12"), (1, 2, None), (4, 9, None)):
            plan = st.Plan(shape, radius, c, storage=storage, anchor_m=m, tune=tune)
            plan.run(x, y, steps)
            torch.cuda.synchronize()
            want = precision.run_scaled(f, c, radius, steps, m, codec)
            assert_bitwise(y.cpu().numpy(), want, f"{storage} m{m} {shape} r{radius} [{plan.describe()}]")
            plan.close()


@pytest.mark.parametrize("radius", [1, 4])
def test_precision_forms_multi_segment_bitwise(torch, st, radius):
    """z-segments of 64 and 128 planes over 200 planes: tile maxima published
    by several segments of one storage tile column, and the exponents staged
    per segment, against the models of both forms."""
    from oracle import precision
    shape = (200, 40, 72)
    c = synth.coefficients(1600 + radius, 3, radius)
    f = synth.sinusoid_grid(1700 + radius, 200, modes=4)[:, :40, :72].copy()
    x = torch.from_numpy(f).cuda()
    y = torch.empty_like(x)
    for storage, codec, model in (("f16", precision.F16, precision.run),
                                  ("bf16-scaled", precision.BF16, precision.run_scaled)):
        want = model(f, c, radius, 6, 3, codec)
        for tune in ("wl=32,nw=16,lz=64", "wl=32,nw=16,lz=128", "wl=64,nw=16,lz=64"):
            plan = st.Plan(shape, radius, c, storage=storage, anchor_m=3, tune=tune)
            plan.run(x, y, 6)
            torch.cuda.synchronize()
            assert_bitwise(y.cpu().numpy(), want, f"{storage} {tune} r{radius} [{plan.describe()}]")
            plan.close()


def test_precision_form_error_and_speed_report(torch, st, oracle_mod):
    """Small sinusoid field: FP16/BF16 error against FP64 stays in the model's range."""
    shape = (64, 64, 128)
    c = synth.coefficients(1300, 3, 4)
    f = synth.sinusoid_grid(1301, 128, modes=8)[:64, :64, :].copy()
    x = torch.from_numpy(f).cuda()
    y = torch.empty_like(x)
    ref = oracle_mod.star_run_f64(f, c, 4, 30)
    for storage, m, tol in (("f16", 10, 1e-3), ("f16", 50, 1e-3), ("bf16", 10, 1e-2)):
        plan = st.Plan(shape, 4, c, storage=storage, anchor_m=m)
        plan.run(x, y, 30)
        torch.cuda.synchronize()
        err = oracle_mod.rel_linf(y.cpu().numpy(), ref)
        assert err <= tol, (storage, m, err)
        plan.close()


def _precision_reference():
    from conftest import golden
    import os
    from conftest import ROOT
    maxabs = None
    with open(os.path.join(ROOT, "tests", "golden", "precision_128cube_r4_1000.txt")) as fh:
        for line in fh:
            if line.startswith("# maxabs"):
                maxabs = float(line.split()[2])
    rows = golden("precision_128cube_r4_1000.txt")
    cells = [(int(r[0]), int(r[1]), int(r[2])) for r in rows]
    vals = np.array([float(r[3]) for r in rows])
    return maxabs, cells, vals


@pytest.mark.parametrize("storage,m,tol", [("f32", 0, TOL_F64), ("f16", 10, 1e-3), ("f16", 50, 1e-3),
                                           ("bf16", 10, 1e-2), ("bf16", 50, 1e-2),
                                           ("f16-scaled", 10, 5e-2), ("bf16-scaled", 10, 5e-1)])
def test_precision_workload_128cube_vs_stored_fp64(torch, st, storage, m, tol):
    """1000 steps of radius 4 on the 128^3 sinusoid grid against the FP64
    oracle values stored for sampled cells (corners included)."""
    maxabs, cells, want = _precision_reference()
    n = 128
    f = synth.sinusoid_grid(4, n)
    c = synth.coefficients(3004, 3, 4)
    x = torch.from_numpy(f).cuda()
    y = torch.empty_like(x)
    plan = st.Plan((n, n, n), 4, c, storage=storage, anchor_m=m)
    plan.run(x, y, 1000)
    torch.cuda.synchronize()
    got = y.cpu().numpy()
    vals = np.array([got[z, yy, xx] for xx, yy, z in cells], dtype=np.float64)
    err = np.max(np.abs(vals - want)) / maxabs
    assert err <= tol, (storage, m, err)
    plan.close()


def test_model_predictions_and_errors(torch, st):
    p2 = st.Plan((4096, 4096), 2, synth.coefficients(3, 2, 2))
    m = p2.model()
    # 2D: no sequential-path term (a lone wavefront's slower issue is in the VALU time)
    assert m["GCell/s"] > 0 and m["hbm_us"] > 0 and m["valu_us"] > 0 and m["plane_us"] == 0
    # more fused steps move fewer bytes per step: higher predicted rate, HBM time per pass unchanged
    assert p2.model("k=4,ly=128")["GCell/s"] > p2.model("k=1,ly=128")["GCell/s"]
    with pytest.raises(ValueError):
        p2.model("k=99")
    p3 = st.Plan((64, 64, 256), 4, synth.coefficients(4, 3, 4))
    m3 = p3.model("k=1,wl=32,lz=64")
    assert m3["GCell/s"] > 0 and m3["plane_us"] > 0
    m3r = p3.model("k=1,rows=1,lz=64")  # the LDS-free layout has no plane latency term
    assert m3r["GCell/s"] > 0 and m3r["hbm_us"] > 0 and m3r["plane_us"] == 0
    # a 64-wide grid fills a quarter of a 256-column strip; four 16-lane
    # rows per wavefront issue a quarter of the wavefronts for the same bytes
    p64 = st.Plan((64, 64, 64), 3, synth.coefficients(6, 3, 3))
    wide, narrow = p64.model("k=1,rows=1,lz=64"), p64.model("k=1,rows=1,lz=64,lpr=16")
    assert narrow["valu_us"] == pytest.approx(wide["valu_us"] / 4)
    assert narrow["hbm_us"] == pytest.approx(wide["hbm_us"])
    p64.close()
    pn = st.Plan((64, 64), 1, synth.coefficients(5, 2, 1), tune="naive")
    with pytest.raises(st.StencilError):
        pn.model()
    for p in (p2, p3, pn):
        p.close()


def test_autotune_prunes_by_model(torch, st, oracle_mod, monkeypatch):
    monkeypatch.setenv("STENCIL_TUNE_TOP", "3")
    monkeypatch.delenv("STENCIL_TUNE_CACHE", raising=False)
    shape, radius = (300, 1100), 3
    c = synth.coefficients(960, 2, radius)
    f = synth.grid_uniform(961, shape)
    x = torch.from_numpy(f).cuda()
    y = torch.empty_like(x)
    p = st.Plan(shape, radius, c)
    rows = p.autotune(x, y)
    assert len(rows) == 3
    timed = {cfg for cfg, _ in rows}
    # the three timed candidates are the model's three best
    worst_timed = min(p.model(cfg)["GCell/s"] for cfg in timed)
    for K in range(1, 6):
        for ly in (64, 96, 128, 192, 256, 384):
            cfg = f"k={K},ly={ly}"
            if cfg not in timed and ly <= shape[0]:
                assert p.model(cfg)["GCell/s"] <= worst_timed + 1e-9, cfg
    p.run(x, y, 6)
    torch.cuda.synchronize()
    assert_bitwise(y.cpu().numpy(), oracle_mod.star_run_f32(f, c, radius, 6), "pruned autotune")
    p.close()
