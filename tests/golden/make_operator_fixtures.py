"""Writes the sampled FP64 oracle outputs used by the full-size (128^3) GPU parity tests.

Calls only the oracle and the seeded input generators. Workload: 128^3 grid,
dx = 100 um, c0 = 1500 m/s, dt = 20 ns, Nt = 740, PML 8 cells; p0 = 24 random
vessels (radius 1-4 voxels, seed 1); rSP 2048 of 16384 pixels (seed 2) and
sHd 2048 patterns (column scramble seed 4, rows seed 5).

Stored (float64 .npz, one file per case):
  forward_*:  columns `cols` of f = C A p0 for all 740 samples
  adjoint_*:  slices z in `zs` (the sensor plane z = 0, two interior slices, one
              slice of the z-PML slab) of A^T C^T y with y = N(0,1) data (seed 5 / 6)
Run: python tests/golden/make_operator_fixtures.py   (about 25 min on 8 cores)
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.sampling import Sampling, apply_c, apply_ct  # noqa: E402
from synthetic import gaussian_data, vessel_phantom  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))
N, NT, P = 128, 740, 8
COLS = np.arange(0, 2048, 64, dtype=np.int64)          # 32 data columns
ZS = np.array([0, 1, 60, 119], dtype=np.int64)         # z slices of the adjoint: sensor plane, interior, z-PML


def main(which=("forward_points", "forward_hadamard", "adjoint_points", "adjoint_hadamard")):
    g = oracle.Grid(N, N, N, dx=100e-6, c0=1500.0, dt=20e-9, nt=NT, pml_size=P)
    op = oracle.WaveOperator(g)
    smps = {"points": Sampling.points(N * N, 2048, 2), "hadamard": Sampling.hadamard(N * N, 2048, 4)}
    p0 = vessel_phantom((N, N, N), P, 24, 1.0, 4.0, 1)
    for case in which:
        t = time.time()
        kind = case.split("_")[1]
        smp = smps[kind]
        path = os.path.join(OUT, f"op128_{case}.npz")
        if case.startswith("forward"):
            f = apply_c(op.forward_planes(p0), smp)
            np.savez_compressed(path, cols=COLS, values=f[:, COLS], norm=np.linalg.norm(f))
        else:
            seed = 5 if kind == "points" else 6
            y = gaussian_data((NT, 2048), seed)
            p = op.adjoint_planes(apply_ct(y, smp, N, N))
            np.savez_compressed(path, zs=ZS, values=p[ZS], norm=np.linalg.norm(p), data_seed=seed)
        print(f"{case}: {time.time() - t:.0f} s -> {path}", flush=True)


if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or ("forward_points", "forward_hadamard", "adjoint_points", "adjoint_hadamard"))
