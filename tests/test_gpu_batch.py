"""GPU parity of the batched form (many grids per call) through the C ABI.

Bar: every grid of a batch is bitwise equal to the oracle's single-precision
result (small grids) and to its own stencil_run (every size), under every
class configuration, with and without the captured graph, on relaunch, and
mixed with grids the batch hands to their own plan (zero steps, FP16
storage).  The full-size mixed batch of 256 grids is checked against
per-grid runs everywhere and against the FP64 oracle on sampled cells.
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


# (numpy shape, radius, steps): 2D and 3D, aligned and ragged rows, sides of
# 1, several strips/tiles/segments, step counts with tail passes, zero steps.
MIXED = [
    ((37, 513), 1, 10), ((1, 1), 2, 3), ((6, 1), 4, 5), ((300, 260), 3, 7),
    ((64, 2048), 2, 11), ((97, 1000), 4, 9), ((130, 1024), 1, 17), ((3, 3), 1, 0),
    ((700, 400), 1, 12),
    ((9, 17, 33), 1, 9), ((4, 5, 6), 3, 4), ((40, 36, 132), 2, 5), ((70, 68, 136), 4, 3),
    ((33, 70, 64), 1, 10), ((1, 1, 1), 2, 2), ((20, 24, 90), 3, 6), ((90, 40, 256), 2, 3),
]

TUNES = [
    None,
    "2d.k=1,3d.k=1",
    "2d.k=3,2d.ly=16,3d.k=2,3d.lz=8",
    "2d.k=8,2d.ly=256,3d.wl=64,3d.nw=12,3d.lz=32",
    "3d.vec=8,3d.wl=64,3d.k=1,streams=1,merge=0",
    "merge=0,2d.k=2",
    "graph=0,streams=2",
    "streams=16,3d.nw=8",
]


def make_inputs(cases, seed0):
    out = []
    for j, (shape, radius, steps) in enumerate(cases):
        c = synth.coefficients(seed0 + 2 * j, len(shape), radius)
        f = synth.grid_uniform(seed0 + 2 * j + 1, shape)
        out.append((f, c, radius, steps))
    return out


@pytest.fixture(scope="module")
def mixed(oracle_mod):
    data = make_inputs(MIXED, 7000)
    want = [oracle_mod.star_run_f32(f, c, r, s) for f, c, r, s in data]
    return data, want


def build(torch, st, data):
    plans = [st.Plan(f.shape, r, c) for f, c, r, s in data]
    ins = [torch.from_numpy(f).cuda() for f, c, r, s in data]
    outs = [torch.full_like(x, float("nan")) for x in ins]
    steps = [s for f, c, r, s in data]
    return plans, ins, outs, steps


def assert_bitwise(got, want, what):
    if not np.array_equal(got, want):
        bad = np.argwhere(got != want)
        raise AssertionError(f"{what}: {len(bad)} cells differ, first at {bad[:5].tolist()}")


@pytest.mark.parametrize("tune", TUNES)
def test_batch_matches_oracle_bitwise(torch, st, mixed, tune):
    data, want = mixed
    plans, ins, outs, steps = build(torch, st, data)
    b = st.Batch(plans, ins, outs, steps, tune=tune)
    desc = b.describe()
    for rep in range(2):  # the replay must clear its counters
        for o in outs:
            o.fill_(float("nan"))
        b.launch()
        torch.cuda.synchronize()
        for j, (o, w) in enumerate(zip(outs, want)):
            assert_bitwise(o.cpu().numpy(), w, f"grid {j} {data[j][0]} r{data[j][2]} "
                                               f"tune={tune} rep={rep}\n{desc}")
    for x, (f, c, r, s) in zip(ins, data):
        assert np.array_equal(x.cpu().numpy(), f)  # inputs are never written
    b.close()


def test_batch_describe_lists_classes(torch, st, mixed):
    data, _ = mixed
    plans, ins, outs, steps = build(torch, st, data)
    b = st.Batch(plans, ins, outs, steps)
    d = b.describe()
    assert "grids=17" in d and "own=1" in d  # the zero-step grid runs by its plan
    assert "2d r=1" in d and "3d r=4" in d
    b.close()


def test_run_batched_repeat_and_change(torch, st, mixed, oracle_mod):
    data, want = mixed
    plans, ins, outs, steps = build(torch, st, data)
    for rep in range(2):
        st.run_batched(plans, ins, outs, steps)
        torch.cuda.synchronize()
        for j, (o, w) in enumerate(zip(outs, want)):
            assert_bitwise(o.cpu().numpy(), w, f"one-shot rep {rep} grid {j}")
    steps2 = [s + 1 for s in steps]
    st.run_batched(plans, ins, outs, steps2)
    torch.cuda.synchronize()
    for j, ((f, c, r, s), o) in enumerate(zip(data, outs)):
        assert_bitwise(o.cpu().numpy(), oracle_mod.star_run_f32(f, c, r, s + 1), f"steps+1 grid {j}")


def test_batch_rejects_shared_memory_and_bad_tune(torch, st):
    data = make_inputs([((40, 50), 1, 3), ((30, 20), 2, 3)], 7100)
    plans, ins, outs, steps = build(torch, st, data)
    with pytest.raises(ValueError):  # one plan twice: its scratch would be shared
        st.Batch([plans[0], plans[0]], [ins[0], ins[0]], [outs[0], torch.empty_like(outs[0])], 3)
    with pytest.raises(ValueError):  # grid 1 writes what grid 0 reads
        st.Batch(plans, ins, [outs[0], ins[0].view(-1)[:600]], steps)
    with pytest.raises(ValueError):  # two outputs overlap
        st.Batch(plans, ins, [outs[0], outs[0].view(-1)[:600]], steps)
    for bad in ("2d.k=0", "streams=99", "nope=1", "3d.wl=48", "graph=2", "2d.ly"):
        with pytest.raises(ValueError):
            st.Batch(plans, ins, outs, steps, tune=bad)
    d3 = make_inputs([((16, 16, 16), 4, 2)], 7200)
    p3, i3, o3, s3 = build(torch, st, d3)
    with pytest.raises(ValueError):  # 4 tile rows cannot hold 2*K*R + 1
        st.Batch(p3, i3, o3, s3, tune="3d.wl=64,3d.nw=4")
    with pytest.raises(ValueError):
        st.Batch(p3, i3, o3, [-1])


def test_batch_hands_lowp_zero_step_and_high_radius_grids_to_their_plans(torch, st):
    f16 = synth.grid_uniform(7301, (9, 70, 72))
    c16 = synth.coefficients(7302, 3, 2)
    plan16 = st.Plan(f16.shape, 2, c16, storage="f16", anchor_m=3)
    x16 = torch.from_numpy(f16).cuda()
    ref16 = torch.empty_like(x16)
    plan16.run(x16, ref16, 7)
    data = make_inputs([((50, 300), 3, 6), ((12, 30, 40), 1, 5), ((20, 20), 1, 0),
                        ((40, 600), 7, 5), ((8, 12, 40), 6, 3)], 7310)
    plans, ins, outs, steps = build(torch, st, data)
    refs = []
    for p, x, s in zip(plans, ins, steps):
        r = torch.empty_like(x)
        p.run(x, r, s)
        refs.append(r)
    out16 = torch.full_like(x16, float("nan"))
    b = st.Batch(plans + [plan16], ins + [x16], outs + [out16], steps + [7])
    b.launch()
    torch.cuda.synchronize()
    assert torch.equal(out16, ref16)
    for j, (o, r) in enumerate(zip(outs, refs)):
        assert torch.equal(o, r), j
    assert torch.equal(outs[2], ins[2])  # zero steps copy
    b.close()


def test_batch_autotune_and_cache(torch, st, mixed, tmp_path, monkeypatch):
    monkeypatch.setenv("STENCIL_TUNE_CACHE", str(tmp_path / "tune.txt"))
    data, want = mixed
    sub = [k for k, d in enumerate(data) if d[3] > 0][:10]
    data = [data[k] for k in sub]
    want = [want[k] for k in sub]
    plans, ins, outs, steps = build(torch, st, data)
    b = st.Batch(plans, ins, outs, steps)
    report = b.autotune()
    assert report.count("\n") >= 10
    torch.cuda.synchronize()
    for j, (o, w) in enumerate(zip(outs, want)):  # autotuning leaves the result in place
        assert_bitwise(o.cpu().numpy(), w, f"after autotune grid {j}")
    assert "by=autotune" in b.describe()
    b.launch()
    torch.cuda.synchronize()
    for j, (o, w) in enumerate(zip(outs, want)):
        assert_bitwise(o.cpu().numpy(), w, f"tuned launch grid {j}")
    b.close()
    lines = (tmp_path / "tune.txt").read_text().splitlines()
    assert any(l.startswith("batch ndim=2") for l in lines)
    assert any(l.startswith("batch ndim=3") for l in lines)
    b2 = st.Batch(plans, ins, outs, steps)
    assert "by=cache" in b2.describe() and "by=default" not in b2.describe()
    b2.close()


@pytest.mark.slow
def test_full_mixed_batch_vs_per_grid_and_sampled_oracle(torch, st, oracle_mod):
    """The 256-grid mixed workload (128 2D grids with sides log-uniform in
    64..4096, 128 3D grids with sides log-uniform in 32..256, radius uniform
    in 1..4, 100 steps) in its default launch configuration."""
    shapes = synth.batch_shapes(5)
    steps = 100
    plans, ins, outs, refs, host = [], [], [], [], []
    for dims, radius, cseed, vseed in shapes:
        shape = tuple(reversed(dims))
        c = synth.coefficients(cseed, len(shape), radius)
        f = synth.grid_uniform(vseed, shape)
        p = st.Plan(shape, radius, c)
        x = torch.from_numpy(f).cuda()
        r = torch.empty_like(x)
        p.run(x, r, steps)
        plans.append(p)
        ins.append(x)
        outs.append(torch.full_like(x, float("nan")))
        refs.append(r)
        host.append((f, c, radius))
    b = st.Batch(plans, ins, outs, steps)
    b.launch()
    torch.cuda.synchronize()
    for j, (o, r) in enumerate(zip(outs, refs)):
        assert torch.equal(o, r), (j, shapes[j])
    # FP64 oracle: the two smallest grids of each dimension in full, the
    # largest 2D grid on sampled cells (corners included)
    for nd in (2, 3):
        idx = sorted((k for k in range(len(host)) if host[k][0].ndim == nd),
                     key=lambda k: host[k][0].size)
        for j in idx[:2]:
            f, c, radius = host[j]
            want = oracle_mod.star_run_f64(f, c, radius, steps)
            assert oracle_mod.rel_linf(outs[j].cpu().numpy(), want) <= TOL_F64, (j, shapes[j])
    j = max((k for k in range(len(host)) if host[k][0].ndim == 2), key=lambda k: host[k][0].size)
    f, c, radius = host[j]
    dims = f.shape[::-1]
    rng = np.random.default_rng(11)
    cells = np.stack([rng.integers(0, n, 4) for n in dims], axis=1)
    cells[0] = 0
    cells[1] = np.array(dims) - 1
    want = oracle_mod.star_sample_f64(f, c, radius, steps, cells)
    got = outs[j].cpu().numpy()
    vals = np.array([got[tuple(cc[::-1])] for cc in cells], dtype=np.float64)
    assert np.max(np.abs(vals - want)) / np.max(np.abs(want)) <= TOL_F64
    b.close()
