"""GPU parity of the TV prox, TV norm, PSNR, power iteration and FISTA/Bregman
against the FP64 oracle, through the C ABI.

Tolerances: prox and reconstructions at fixed iteration counts within 1e-4
relative L2; scalars (TV, PSNR, L) within FP32 rounding of their inputs.
"""

import math
import os

import numpy as np
import pytest

import oracle
from oracle.metrics import eval_region, psnr
from oracle.solvers import FistaLog, MeasuredOperator, bregman, fista, power_iteration
from oracle.tv import prox_tv_pos, tv_value
from gpu_cases import (empty, gaussian_data, gaussian_volume, gpu_plan, oracle_grid, oracle_sampling, phantom,
                       rel_l2, to_dev, to_host)

pytestmark = pytest.mark.gpu

TOL_RECON = 1e-4
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _fixture(name):
    path = os.path.join(GOLDEN, f"{name}.npz")
    assert os.path.exists(path), f"committed fixture {path} is missing"
    return np.load(path)


def _oracle_dual_to_gpu(y, bc):
    if bc == "dirichlet":
        return y[:, :-1, :-1, :-1]
    return y


@pytest.mark.parametrize("bc", ["neumann", "dirichlet"])
def test_tv_prox_matches_oracle_with_warm_start(bc):
    from paper_1605_00133_amd import pat as P
    n = 32
    plan = gpu_plan(n, 2, oracle_sampling("full", n))
    v = phantom(n) + 0.1 * gaussian_volume((n, n, n), 4)
    alpha = 0.05
    q1, y1 = prox_tv_pos(v, alpha, 50, bc)
    q2, y2 = prox_tv_pos(v * 0.9, alpha, 30, bc, dual=y1)
    nd = P.pat_tv_dual_floats(plan.grid, bc)
    dual = to_dev(np.zeros(nd))
    q = empty(plan.vol_shape)
    P.pat_tv_prox(plan, to_dev(v), q, alpha, 50, bc, dual)
    e1 = rel_l2(to_host(q), q1)
    ed = rel_l2(to_host(dual).reshape((3,) + ((n + 1,) * 3 if bc == "dirichlet" else (n,) * 3)),
                _oracle_dual_to_gpu(y1, bc))
    vv = to_dev(v * 0.9)
    P.pat_tv_prox(plan, vv, vv, alpha, 30, bc, dual)          # in place, warm start
    e2 = rel_l2(to_host(vv), q2)
    print(f"prox {bc}: q {e1:.2e}, dual {ed:.2e}, warm-started in-place q {e2:.2e}")
    assert e1 < TOL_RECON and ed < TOL_RECON and e2 < TOL_RECON


@pytest.mark.parametrize("bc", ["neumann", "dirichlet"])
def test_tv_norm_matches_oracle(bc):
    from paper_1605_00133_amd import pat as P
    n = 32
    plan = gpu_plan(n, 2, oracle_sampling("full", n))
    x = phantom(n) + 0.05 * gaussian_volume((n, n, n), 6)
    x32 = x.astype(np.float32).astype(np.float64)
    got = P.pat_tv_norm(plan, to_dev(x), bc)
    ref = tv_value(x32, bc)
    print(f"TV {bc}: {got!r} vs {ref!r}")
    assert abs(got - ref) / ref < 1e-6


def test_psnr_matches_oracle():
    from paper_1605_00133_amd import pat as P
    n = 32
    plan = gpu_plan(n, 2, oracle_sampling("full", n))
    a = phantom(n)
    b = a + 0.05 * gaussian_volume((n, n, n), 7)
    a32 = a.astype(np.float32).astype(np.float64)
    b32 = b.astype(np.float32).astype(np.float64)
    got = P.pat_psnr(plan, to_dev(b), to_dev(a))
    ref = psnr(b32, a32, eval_region(oracle_grid(n, 2)))
    print(f"PSNR {got} vs {ref}")
    assert abs(got - ref) < 1e-9 * abs(ref)
    assert P.pat_psnr(plan, to_dev(a), to_dev(a)) == float("inf")


def test_psnr_evaluation_region_worked_example():
    """The GPU's evaluation region, pinned by hand (independently of the oracle's eval_region).

    16^3 grid, P = 2: z in [1, nz - 2P) = [1, 12), y and x in [2, 14), N = 11 * 12 * 12 = 1584.
    Large values on the sensor layer, the first z-PML layer, deep in the z-PML and one cell
    into each lateral PML face would set the maximum if they were inside. Inside, p differs from
    p0 by 0.5 at the first corner and 0.25 at the last: PSNR = -10 log10(0.3125 / 1584).
    """
    from paper_1605_00133_amd import pat as P
    n = 16
    plan = gpu_plan(n, 2, oracle_sampling("full", n), pml=2)
    p0 = np.zeros((n, n, n))
    p0[5, 7, 7] = 1.0
    p0[0, 8, 8] = 9.0
    p0[13, 8, 8] = 9.0
    p = p0.copy()
    p[0, 8, 8] = p[13, 8, 8] = 0.0
    p[0, 7, 7] = 50.0
    p[12, 7, 7] = 40.0
    p[15, 7, 7] = 30.0
    p[5, 1, 7] = p[5, 14, 7] = p[5, 7, 1] = p[5, 7, 14] = 20.0
    p[1, 2, 2] = 0.5
    p[11, 13, 13] = 0.25
    got = P.pat_psnr(plan, to_dev(p), to_dev(p0))
    ref = -10 * math.log10(0.3125 / 1584)
    print(f"PSNR region example: {got!r} vs {ref!r}")
    assert abs(got - ref) < 1e-9 * ref


def test_power_iteration_matches_oracle():
    from paper_1605_00133_amd import pat as P
    n, nt = 32, 190
    smp = oracle_sampling("points", n)
    g = oracle_grid(n, nt)
    op = MeasuredOperator(oracle.WaveOperator(g), smp)
    x0 = gaussian_volume((n, n, n), 8)
    ref = power_iteration(op, x0, 6)
    plan = gpu_plan(n, nt, smp)
    got = P.pat_power_iteration(plan, to_dev(x0), 6)
    print(f"L: GPU {got} vs oracle {ref}")
    assert abs(got - ref) / ref < 1e-5


def _small_problem(kind="points"):
    n, nt = 32, 190
    smp = oracle_sampling(kind, n)
    g = oracle_grid(n, nt)
    op = MeasuredOperator(oracle.WaveOperator(g), smp)
    p0 = phantom(n)
    clean = op.forward(p0)
    f = clean + 0.01 * np.abs(clean).max() * gaussian_data(clean.shape, 3)
    L = power_iteration(op, gaussian_volume((n, n, n), 8), 20)
    return n, nt, smp, op, p0, f, L


@pytest.mark.parametrize("restart", [False, True])
def test_fista_tv_matches_oracle(restart):
    """The small workload: 10 FISTA iterations of TV+ (lambda = 1e-3), Dirichlet TV, 50 PDHG steps."""
    from paper_1605_00133_amd import pat as P
    n, nt, smp, op, p0, f, L = _small_problem()
    lam = 1e-3
    log = FistaLog()
    ref, _, _ = fista(op, f, lam, L, 10, 50, "dirichlet", restart=restart, log=log)
    plan = gpu_plan(n, nt, smp)
    p = empty(plan.vol_shape)
    out = P.pat_reconstruct(plan, to_dev(f), p, lam, L, 1, 10, 50, "dirichlet", restart=restart,
                            p_ref=to_dev(p0))
    err = rel_l2(to_host(p), ref)
    print(f"FISTA restart={restart}: rel L2 {err:.2e}; flags GPU {list(out['flags'])} oracle {log.flags}")
    print("energies GPU", out["energy"], "oracle", np.array(log.energy))
    assert list(out["flags"]) == log.flags
    assert np.allclose(out["energy"], log.energy, rtol=1e-4)
    assert err < TOL_RECON
    assert np.all(np.isfinite(out["psnr"]))


def test_bregman_matches_oracle_and_residual_decreases():
    from paper_1605_00133_amd import pat as P
    n, nt, smp, op, p0, f, L = _small_problem("hadamard")
    lam = 1e-2
    ref, res = bregman(op, f, lam, L, 3, 4, 30, "dirichlet")
    plan = gpu_plan(n, nt, smp)
    p = empty(plan.vol_shape)
    out = P.pat_reconstruct(plan, to_dev(f), p, lam, L, 3, 4, 30, "dirichlet")
    err = rel_l2(to_host(p), ref)
    print(f"Bregman 3x4: rel L2 {err:.2e}; residuals GPU {out['bregman_residual']} oracle {res}")
    assert err < TOL_RECON
    assert np.allclose(out["bregman_residual"], res, rtol=1e-4)
    assert np.all(np.diff(out["bregman_residual"]) < 0)


def test_fista_restart_branch_matches_oracle():
    """The restart + backtracking branch of App. B on the GPU against the oracle.

    The oracle run is stored by tests/golden/make_solver_fixtures.py (restart32_points): the
    small workload with L underestimated 3x, so the energy rises and the branch runs in most
    iterations (plain gradient step from the previous iterate, halvings, t reset). The data
    are recomputed here by the oracle with the stored sigma. Flags must be identical, with
    at least one halving; energies and the reconstruction within 1e-4.
    """
    from paper_1605_00133_amd import pat as P
    fx = _fixture("restart32_points")
    n, nt = 32, 190
    smp = oracle_sampling("points", n)
    op = MeasuredOperator(oracle.WaveOperator(oracle_grid(n, nt)), smp)
    p0 = phantom(n)
    clean = op.forward(p0)
    f = clean + float(fx["sigma"]) * gaussian_data(clean.shape, 3)
    plan = gpu_plan(n, nt, smp)
    p = empty(plan.vol_shape)
    out = P.pat_reconstruct(plan, to_dev(f), p, float(fx["lam"]), float(fx["L"]), 1, 10, 50, "dirichlet",
                            restart=True)
    err = rel_l2(to_host(p), fx["x"])
    print(f"FISTA forced restarts: rel L2 {err:.2e}; flags GPU {list(out['flags'])} oracle {list(fx['flags'])}")
    print("energies GPU", out["energy"], "oracle", fx["energy"])
    assert list(out["flags"]) == list(fx["flags"])
    assert max(fx["flags"]) >= 2
    assert np.allclose(out["energy"], fx["energy"], rtol=1e-4)
    assert np.allclose(out["residual"], fx["residual"], rtol=1e-4)
    assert err < TOL_RECON
