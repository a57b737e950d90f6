"""Writes fp64_<case>.txt: FP64 oracle values of the full-size workloads at
their full step counts, on sampled cells.

Cases (grid seed / coefficient seed as the benchmark draws them):
  2d16k_r{1..4}  2D star, radius R, 16384^2 uniform [0,1) grid (seed 1),
                 coefficients seed 1000 + R, 1000 steps;
  3d512_r{1..4}  3D star, radius R, 512^3 uniform [0,1) grid (seed 2),
                 coefficients seed 2000 + R, 200 steps;
  3d768sin_r4    3D star, radius 4, 768^3 seeded sinusoid grid (seed 4: 8
                 low-frequency modes plus 1e-3 noise), coefficients seed
                 3004, 1000 steps.
All with the clamp boundary (Eq. (1) of Sec. IV.A, Sec. III.B), 1000 steps
being the iteration count of Sec. IV.C.

Each file keeps max |f| and the sum of f over the whole grid (the normaliser
of the normwise relative L-infinity error, and the conservation sum) and
the values at sampled cells: every corner with its neighbours one and two
cells inward, cells within 16 of a face, cells on the lines x, y (, z) in
{63, 64, 127, 128, 255, 256} (typical tile and segment seams), and cells
drawn uniformly (numpy's PCG64 with a fixed seed).

Only the oracle and the input generators are called.

  python tests/golden/make_fullsize_reference.py [case ...] [--threads N]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle  # noqa: E402
from paper_2002_05983_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
SEAMS = (63, 64, 127, 128, 255, 256)


def cases():
    out = {}
    for r in (1, 2, 3, 4):
        out[f"2d16k_r{r}"] = dict(ndim=2, dims=(16384, 16384), radius=r, steps=1000,
                                  grid=("uniform", 1), coef=1000 + r, random=900)
    for r in (1, 2, 3, 4):
        out[f"3d512_r{r}"] = dict(ndim=3, dims=(512, 512, 512), radius=r, steps=200,
                                  grid=("uniform", 2), coef=2000 + r, random=768)
    out["3d768sin_r4"] = dict(ndim=3, dims=(768, 768, 768), radius=4, steps=1000,
                              grid=("sinusoid", 4), coef=3004, random=3840)
    return out


def sample_cells(dims, n_random: int, seed: int) -> np.ndarray:
    """Sampled (x, y[, z]) cells, duplicates removed, in a fixed order."""
    ndim = len(dims)
    rng = np.random.default_rng(seed)
    pts = []
    # corners and the cells one and two steps inward along every axis
    for corner in np.ndindex(*([2] * ndim)):
        for inward in range(3):
            pts.append([inward if b == 0 else n - 1 - inward for b, n in zip(corner, dims)])
            for a in range(ndim):
                p = [0 if b == 0 else n - 1 for b, n in zip(corner, dims)]
                p[a] = inward if corner[a] == 0 else dims[a] - 1 - inward
                pts.append(p)
    # within 16 cells of a face
    for a in range(ndim):
        for side in (0, 1):
            for _ in range(24):
                p = [int(rng.integers(0, n)) for n in dims]
                d = int(rng.integers(0, 16))
                p[a] = d if side == 0 else dims[a] - 1 - d
                pts.append(p)
    # on seam lines
    for a in range(ndim):
        for s in SEAMS:
            if s < dims[a]:
                for _ in range(4):
                    p = [int(rng.integers(0, n)) for n in dims]
                    p[a] = s
                    pts.append(p)
    # uniform
    for _ in range(n_random):
        pts.append([int(rng.integers(0, n)) for n in dims])
    seen, out = set(), []
    for p in pts:
        t = tuple(p)
        if t not in seen:
            seen.add(t)
            out.append(t)
    return np.array(out, dtype=np.int64)


def make_grid(spec):
    kind, seed = spec["grid"]
    shape = spec["dims"][::-1]
    if kind == "uniform":
        return synth.grid_uniform(seed, shape)
    return synth.sinusoid_grid(seed, spec["dims"][0])


def write_case(name: str, spec, threads: int):
    t0 = time.time()
    f = make_grid(spec)
    c = synth.coefficients(spec["coef"], spec["ndim"], spec["radius"])
    ref = oracle.star_run_f64(f, c, spec["radius"], spec["steps"], threads=threads)
    del f
    cells = sample_cells(spec["dims"], spec["random"], seed=hash_seed(name))
    vals = ref[tuple(cells[:, a] for a in range(spec["ndim"] - 1, -1, -1))]
    maxabs = float(np.abs(ref).max())
    total = float(ref.sum(dtype=np.float64))
    secs = time.time() - t0
    dims_s = "x".join(str(d) for d in spec["dims"])
    grid = ("uniform [0,1) (seed %d)" % spec["grid"][1] if spec["grid"][0] == "uniform"
            else "sinusoid recipe (seed %d)" % spec["grid"][1])
    path = os.path.join(HERE, f"fp64_{name}.txt")
    with open(path + ".tmp", "w") as fh:
        fh.write(f"# FP64 oracle (Eq. (1), clamp boundary): {spec['ndim']}D star radius "
                 f"{spec['radius']}, {dims_s} grid {grid},\n")
        fh.write(f"# coefficients seed {spec['coef']}, after {spec['steps']} steps.  Written by "
                 f"tests/golden/make_fullsize_reference.py {name}\n")
        fh.write(f"# ({secs:.0f} s with {threads} threads).\n")
        fh.write(f"# dims {' '.join(str(d) for d in spec['dims'])}\n")
        fh.write(f"# radius {spec['radius']}\n# steps {spec['steps']}\n")
        fh.write(f"# grid {spec['grid'][0]} {spec['grid'][1]}\n# coef_seed {spec['coef']}\n")
        fh.write(f"# maxabs {maxabs!r}\n# sum {total!r}\n")
        fh.write("# columns: x y" + (" z" if spec["ndim"] == 3 else "") + " value\n")
        for p, v in zip(cells, vals):
            fh.write(" ".join(str(int(q)) for q in p) + f" {float(v)!r}\n")
    os.replace(path + ".tmp", path)
    print(f"{name}: {len(cells)} cells, maxabs {maxabs:.6g}, {secs:.0f} s", flush=True)


def hash_seed(name: str) -> int:
    """A fixed per-case seed for the cell draw (independent of Python's hash)."""
    h = 1469598103934665603
    for ch in name.encode():
        h = ((h ^ ch) * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*")
    ap.add_argument("--threads", type=int, default=0)
    args = ap.parse_args()
    table = cases()
    names = args.cases or list(table)
    threads = args.threads or oracle.max_threads()
    for name in names:
        write_case(name, table[name], threads)


if __name__ == "__main__":
    main()
