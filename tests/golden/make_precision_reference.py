"""Writes precision_128cube_r4_1000.txt: FP64 oracle values of a reduced
precision-form workload, on sampled cells.

Workload: a 128^3 grid from the seeded sinusoid recipe (8 low-frequency
modes plus 1e-3 uniform noise, seed 4), 3D star stencil of radius 4 with
seeded coefficients (seed 3004) summing to 1, clamp boundary, 1000 steps.
The FP64 oracle runs the full grid; the file keeps max |f| over the grid
(the rel-L-infinity normaliser) and the values at 8 corners plus 248 cells
drawn from SplitMix64 stream 77.

Only the oracle and the input generators are called.

  python tests/golden/make_precision_reference.py
"""
from __future__ import annotations

import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import oracle  # noqa: E402
from paper_2002_05983_amd import synth  # noqa: E402

N, RADIUS, STEPS = 128, 4, 1000
GRID_SEED, COEF_SEED, CELL_SEED = 4, 3004, 77
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "precision_128cube_r4_1000.txt")


def sample_cells(n: int) -> np.ndarray:
    """(x, y, z) cells: the 8 corners, then 248 drawn uniformly."""
    corners = [(x, y, z) for z in (0, n - 1) for y in (0, n - 1) for x in (0, n - 1)]
    d = synth.uniform01_f64(CELL_SEED, 3 * 248)
    drawn = (d.reshape(248, 3) * n).astype(np.int64)
    return np.vstack([np.array(corners, dtype=np.int64), drawn])


def main():
    f = synth.sinusoid_grid(GRID_SEED, N)
    c = synth.coefficients(COEF_SEED, 3, RADIUS)
    ref = oracle.star_run_f64(f.astype(np.float64), c, RADIUS, STEPS)
    cells = sample_cells(N)
    with open(OUT, "w") as fh:
        fh.write("# FP64 oracle (Eq. (1), clamp boundary) after 1000 steps of a radius-4 3D star\n")
        fh.write("# stencil on the 128^3 seeded sinusoid grid (seed 4, coefficients seed 3004),\n")
        fh.write("# written by tests/golden/make_precision_reference.py.\n")
        fh.write(f"# maxabs {float(np.abs(ref).max())!r}\n")
        fh.write("# columns: x y z value\n")
        for x, y, z in cells:
            fh.write(f"{x} {y} {z} {float(ref[z, y, x])!r}\n")


if __name__ == "__main__":
    main()
