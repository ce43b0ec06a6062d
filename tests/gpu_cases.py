"""Shared set-up for the GPU parity tests: seeded inputs, plans and oracle twins."""

import numpy as np

import oracle
from oracle.sampling import Sampling
from synthetic import vessel_phantom, gaussian_volume, gaussian_data


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def oracle_grid(n, nt, pml=8, dx=100e-6, c0=1500.0, dt=20e-9):
    return oracle.Grid(n, n, n, dx=dx, c0=c0, dt=dt, nt=nt, pml_size=pml)


def oracle_sampling(kind, n, mc=None, seed=2):
    npix = n * n
    if kind == "full":
        return Sampling.full(npix)
    if kind == "points":
        return Sampling.points(npix, mc or npix // 4, seed)
    return Sampling.hadamard(npix, mc or npix // 8, seed)


def gpu_plan(n, nt, smp, pml=8, dx=100e-6, c0=1500.0, dt=20e-9):
    from paper_1605_00133_amd import pat as P
    g = P.make_grid(n, n, n, dx, c0, dt, nt, pml)
    return P.Plan(g, smp.kind, smp.mc, smp.idx, smp.perm)


def phantom(n, pml=8, seed=1):
    nv, rmax = (6, 2.0) if n <= 32 else (24, 4.0)
    return vessel_phantom((n, n, n), pml, nv, 1.0, rmax, seed)


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def empty(shape):
    import torch
    return torch.empty(shape, dtype=torch.float32, device="cuda:0")


__all__ = ["rel_l2", "oracle_grid", "oracle_sampling", "gpu_plan", "phantom", "to_dev", "to_host", "empty",
           "gaussian_volume", "gaussian_data"]
