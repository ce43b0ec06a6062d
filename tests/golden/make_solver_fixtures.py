"""Writes FP64 oracle results of the reconstruction used by the GPU solver parity tests.

Calls only the oracle and the seeded input generators (synthetic/). Every case
draws its phantom, mask and noise from the seeds below; data are
f = C A p0 + sigma * N(0, 1), sigma = 0.01 max |C A p0| (the oracle's sigma is
stored, and the GPU side scales its noise by the same number).

Cases (float64 .npz, one file each):
  restart32_points   32^3, Nt = 190, rSP 256 of 1024 (seed 2), 6 vessels (seed 1),
                     noise seed 3; L = (20 power steps from N(0,1) seed 8) / 3, an
                     underestimate that makes the energy rise, so the restart and
                     backtracking branch of App. B runs; TV+ (lambda = 1e-3,
                     Dirichlet), 10 FISTA iterations, 50 PDHG steps each.
                     Stored: x, L, sigma, flags, energies, residual norms.
  recon128_points    128^3, Nt = 740, rSP 2048 of 16384 (seed 2), 24 vessels of
  recon128_hadamard  radius 1-4 (seed 1), sHd 2048 rows (seeds 4/5), noise seed 3;
                     one Bregman step of 2 FISTA iterations (50 PDHG steps,
                     Dirichlet, restart on), L = 4.5 and lambda = 5e-3 as fixed
                     step and weight parameters (parity does not depend on their
                     values: both sides use the same ones). Stored: z-slices `zs`
                     of x, |x|, sigma, flags, energies, residual norms, the
                     Bregman residual.
Run: python tests/golden/make_solver_fixtures.py [case ...]
     (restart32: about 2 min on 8 cores; each 128^3 case: about 30 min)
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle.sampling import Sampling  # noqa: E402
from oracle.solvers import FistaLog, MeasuredOperator, bregman, fista, power_iteration  # noqa: E402
from synthetic import gaussian_data, gaussian_volume, vessel_phantom  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))
ZS128 = np.array([0, 1, 40, 60, 100, 111], dtype=np.int64)
CASES = ("restart32_points", "recon128_points", "recon128_hadamard")


def _data(op, p0):
    clean = op.forward(p0)
    sigma = 0.01 * float(np.abs(clean).max())
    return clean + sigma * gaussian_data(clean.shape, 3), sigma


def restart32(path):
    n, nt, P = 32, 190, 8
    g = oracle.Grid(n, n, n, dx=100e-6, c0=1500.0, dt=20e-9, nt=nt, pml_size=P)
    op = MeasuredOperator(oracle.WaveOperator(g), Sampling.points(n * n, 256, 2))
    p0 = vessel_phantom((n, n, n), P, 6, 1.0, 2.0, 1)
    f, sigma = _data(op, p0)
    L = power_iteration(op, gaussian_volume((n, n, n), 8), 20) / 3.0
    log = FistaLog()
    x, _, _ = fista(op, f, 1e-3, L, 10, 50, "dirichlet", restart=True, log=log)
    np.savez_compressed(path, x=x, L=L, lam=1e-3, sigma=sigma, flags=np.array(log.flags),
                        energy=np.array(log.energy), residual=np.array(log.residual))
    return log.flags


def recon128(path, kind):
    n, nt, P = 128, 740, 8
    g = oracle.Grid(n, n, n, dx=100e-6, c0=1500.0, dt=20e-9, nt=nt, pml_size=P)
    smp = Sampling.points(n * n, 2048, 2) if kind == "points" else Sampling.hadamard(n * n, 2048, 4)
    op = MeasuredOperator(oracle.WaveOperator(g), smp)
    p0 = vessel_phantom((n, n, n), P, 24, 1.0, 4.0, 1)
    f, sigma = _data(op, p0)
    log = FistaLog()
    x, res = bregman(op, f, 5e-3, 4.5, 1, 2, 50, "dirichlet", restart=True, log=log)
    np.savez_compressed(path, zs=ZS128, values=x[ZS128], norm=np.linalg.norm(x), L=4.5, lam=5e-3, sigma=sigma,
                        flags=np.array(log.flags), energy=np.array(log.energy),
                        residual=np.array(log.residual), bregman_residual=np.array(res))
    return log.flags


def main(which=CASES):
    for case in which:
        t = time.time()
        path = os.path.join(OUT, f"{case}.npz")
        if case == "restart32_points":
            flags = restart32(path)
        else:
            flags = recon128(path, case.split("_")[1])
        print(f"{case}: flags {list(flags)}, {time.time() - t:.0f} s -> {path}", flush=True)


if __name__ == "__main__":
    main(tuple(sys.argv[1:]) or CASES)
