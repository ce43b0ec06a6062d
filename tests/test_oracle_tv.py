"""Pins of the oracle's discrete TV and positivity-constrained TV prox (CPU only)."""

import math

import numpy as np
import pytest
from scipy.optimize import lsq_linear

from oracle.tv import grad, div, tv_value, prox_tv_pos


def test_tv_hand_example():
    """2x2x2 volume with a single voxel of value 1 at the origin, worked by hand (App. A)."""
    p = np.zeros((2, 2, 2))
    p[0, 0, 0] = 1.0
    # Neumann: only voxel (0,0,0) has nonzero forward differences (-1, -1, -1)
    assert abs(tv_value(p, "neumann") - math.sqrt(3.0)) < 1e-15
    # Dirichlet adds the jumps to zero at the three low faces: three padded voxels with |1|
    assert abs(tv_value(p, "dirichlet") - (math.sqrt(3.0) + 3.0)) < 1e-15


def test_tv_constant_neumann_zero_dirichlet_surface():
    p = np.full((4, 5, 6), 2.0)
    assert tv_value(p, "neumann") == 0.0
    # Dirichlet on a constant cube: each boundary face contributes the jump of 2 per voxel,
    # except voxels on the low faces combine up to three jumps in one isotropic norm.
    assert tv_value(p, "dirichlet") > 0.0


def test_div_is_negative_adjoint_of_grad():
    rng = np.random.default_rng(0)
    p = rng.standard_normal((5, 6, 7))
    y = rng.standard_normal((3, 5, 6, 7))
    assert abs(np.vdot(grad(p), y) + np.vdot(p, div(y))) < 1e-12


@pytest.mark.parametrize("bc", ["neumann", "dirichlet"])
def test_prox_alpha_zero_is_clip(bc):
    v = np.random.default_rng(1).standard_normal((6, 6, 6))
    q, _ = prox_tv_pos(v, 0.0, 20, bc)
    assert np.allclose(q, np.maximum(v, 0.0), atol=1e-12)


def test_prox_constant_nonnegative_neumann_is_identity():
    v = np.full((5, 5, 5), 0.7)
    q, _ = prox_tv_pos(v, 0.3, 50, "neumann")
    assert np.allclose(q, v, atol=1e-12)


def test_prox_large_alpha():
    v = np.random.default_rng(2).standard_normal((4, 4, 4)) + 0.5
    # the accelerated PDHG primal error decays like 1/n: 2e-4 after 3e3 steps, 2e-5 after 3e4
    qn, _ = prox_tv_pos(v, 1e3, 30000, "neumann")
    assert np.allclose(qn, max(0.0, v.mean()), atol=5e-5)
    qd, _ = prox_tv_pos(v, 1e3, 30000, "dirichlet")
    assert np.allclose(qd, 0.0, atol=5e-5)


def _tv1d_prox_reference(v, alpha):
    """1D TV denoising (Neumann) through its box-constrained dual, solved by scipy's lsq_linear."""
    n = len(v)
    D = np.zeros((n - 1, n))
    D[np.arange(n - 1), np.arange(n - 1)] = -1.0
    D[np.arange(n - 1), np.arange(1, n)] = 1.0
    res = lsq_linear(D.T, v, bounds=(-alpha, alpha), tol=1e-14, lsmr_tol="auto", max_iter=10000)
    return v - D.T @ res.x


def test_prox_1d_line_matches_direct_solver():
    """On an Nx x 1 x 1 line the isotropic TV is the 1D TV; the 1D prox of TV + (q >= 0) is clip(prox_TV)."""
    rng = np.random.default_rng(3)
    v = np.cumsum(rng.standard_normal(24)) * 0.3 + 0.8    # clip active on part of the line
    alpha = 0.4
    ref = np.maximum(_tv1d_prox_reference(v, alpha), 0.0)
    assert 0 < np.count_nonzero(ref) < len(ref)
    # primal error of the accelerated PDHG decays like 1/n (6.8e-5 at 2e4 steps, 1.4e-5 at 1e5)
    q, _ = prox_tv_pos(v.reshape(1, 1, -1), alpha, 100000, "neumann")
    assert np.max(np.abs(q.ravel() - ref)) < 2e-5


@pytest.mark.parametrize("bc", ["neumann", "dirichlet"])
def test_prox_kkt_conditions(bc):
    """At convergence: |y_i| <= alpha, q = max(0, v + div y), <y, grad q> = alpha TV(q)."""
    rng = np.random.default_rng(4)
    v = rng.standard_normal((6, 7, 8)) * 0.5 + 0.3
    alpha = 0.15
    # the stationarity residual decays like 1/n: 4.5e-4 after 5e3 steps, 4.5e-5 after 5e4
    q, y = prox_tv_pos(v, alpha, 50000, bc)
    if bc == "dirichlet":
        qp = np.pad(q, 1)
        vp = np.pad(v, 1)
        inner = (slice(1, -1),) * 3
    else:
        qp, vp, inner = q, v, (slice(None),) * 3
    nrm = np.sqrt((y * y).sum(axis=0))
    assert nrm.max() <= alpha * (1 + 1e-6)
    assert np.max(np.abs(q - np.maximum(0.0, vp + div(y))[inner])) < 1e-4
    assert abs(np.vdot(y, grad(qp)) - alpha * tv_value(q, bc)) < 1e-6 * max(1.0, alpha * tv_value(q, bc))
