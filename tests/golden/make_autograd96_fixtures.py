"""Writes the FP64 oracle gradients used by the 96^3 differentiation test (GPU).

Calls only the oracle and the seeded input generators. Workload: 96^3 grid incl.
an 8-cell PML, dx = 100 um, c0 = 1500 m/s, dt = 20 ns, Nt = 560, random 25 %
single points of the 96 x 96 plane (2304 of 9216, seed 2); a batch of four:
sample i has data b_i = C A q_i + sigma_i N(0, 1) (q_i: 24 random vessels of
radius 1-4, seed 20 + i; sigma_i = 0.01 max |C A q_i|; noise seed 40 + i) and
is evaluated at p_i (24 vessels, seed 30 + i). Stored per sample: z-slices `zs`
(the sensor plane, two interior slices, one z-PML slice) and the norm of the
gradient of 1/2 ||C A p_i - b_i||^2, i.e. A^T C^T (C A p_i - b_i), and sigma_i.
Run: python tests/golden/make_autograd96_fixtures.py   (about 20 min on 8 cores)
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
N, NT, P, MC = 96, 560, 8, 2304
ZS = np.array([0, 1, 40, 87], dtype=np.int64)
BATCH = 4


def main():
    g = oracle.Grid(N, N, N, dx=100e-6, c0=1500.0, dt=20e-9, nt=NT, pml_size=P)
    op = oracle.WaveOperator(g)
    smp = Sampling.points(N * N, MC, 2)
    vals, norms, sigmas = [], [], []
    for i in range(BATCH):
        t = time.time()
        q = vessel_phantom((N, N, N), P, 24, 1.0, 4.0, 20 + i)
        clean = apply_c(op.forward_planes(q), smp)
        sigma = 0.01 * float(np.abs(clean).max())
        b = clean + sigma * gaussian_data(clean.shape, 40 + i)
        p = vessel_phantom((N, N, N), P, 24, 1.0, 4.0, 30 + i)
        r = apply_c(op.forward_planes(p), smp) - b
        grad = op.adjoint_planes(apply_ct(r, smp, N, N))
        vals.append(grad[ZS])
        norms.append(np.linalg.norm(grad))
        sigmas.append(sigma)
        print(f"sample {i}: {time.time() - t:.0f} s", flush=True)
    path = os.path.join(OUT, "grad96_points.npz")
    np.savez_compressed(path, zs=ZS, values=np.array(vals), norms=np.array(norms), sigmas=np.array(sigmas))
    print(f"-> {path}", flush=True)


if __name__ == "__main__":
    main()
