"""Pins of the oracle's FISTA, Bregman and power iteration (CPU only)."""

import numpy as np
import pytest
from scipy.optimize import nnls

from oracle import Grid, Sampling
from oracle.dense import DenseOperator
from oracle.solvers import FistaLog, bregman, fista, power_iteration
from oracle.tv import div, grad, tv_value


class MatOp:
    """x -> M x on a small volume, same interface as the wave-based operator."""

    def __init__(self, M, shape):
        self.M = M
        self.in_shape = shape
        self.out_shape = (M.shape[0],)

    def forward(self, x):
        return self.M @ np.asarray(x).ravel()

    def adjoint(self, r):
        return (self.M.T @ r).reshape(self.in_shape)


def _problem(shape=(4, 5, 6), rows=200, noise=0.3, seed=0):
    rng = np.random.default_rng(seed)
    M = rng.standard_normal((rows, int(np.prod(shape)))) / np.sqrt(rows)
    p0 = np.zeros(shape)
    p0[1:3, 1:4, 2:5] = 1.0
    d = M @ p0.ravel() + noise * rng.standard_normal(rows)
    return MatOp(M, shape), d, np.linalg.norm(M, 2) ** 2


def test_fista_without_tv_is_nonnegative_least_squares():
    """lam = 0 makes the prox an exact clip: FISTA must reach scipy's NNLS solution."""
    op, d, L = _problem()
    ref, _ = nnls(op.M, d)
    assert (ref == 0).sum() > 10                     # constraints are active
    log = FistaLog()
    x, r, _ = fista(op, d, 0.0, L, 400, 1, "neumann", log=log)
    assert np.linalg.norm(x.ravel() - ref) / np.linalg.norm(ref) < 1e-10
    assert np.allclose(r, op.forward(x) - d, atol=1e-12)   # residual formed by linearity is exact


def _cp_full_problem(op, d, lam, bc, n_iter):
    """Chambolle-Pock on min_{x>=0} 1/2||Mx - d||^2 + lam TV(x) with K = [M; grad] (independent solver)."""
    shape = op.in_shape
    pad = bc == "dirichlet"
    M = op.M
    L = np.linalg.norm(M, 2) ** 2
    tau = sig = 0.99 / np.sqrt(L + 12.0)
    g2 = (lambda x: grad(np.pad(x, 1))) if pad else grad
    g2t = (lambda y: -div(y)[1:-1, 1:-1, 1:-1]) if pad else (lambda y: -div(y))
    x = np.zeros(shape)
    xb = x.copy()
    y1 = np.zeros(M.shape[0])
    y2 = np.zeros((3,) + tuple(s + 2 * pad for s in shape))
    for _ in range(n_iter):
        y1 = (y1 + sig * (M @ xb.ravel()) - sig * d) / (1.0 + sig)
        y2 = y2 + sig * g2(xb)
        y2 = y2 / np.maximum(1.0, np.sqrt((y2 * y2).sum(axis=0)) / lam)
        xn = np.maximum(0.0, x - tau * ((M.T @ y1).reshape(shape) + g2t(y2)))
        xb = 2.0 * xn - x
        x = xn
    return x


@pytest.mark.parametrize("bc", ["neumann", "dirichlet"])
def test_fista_tv_reaches_cp_minimiser(bc):
    op, d, L = _problem(shape=(3, 4, 5), rows=120, noise=0.1)
    lam = 0.05
    E = lambda x: 0.5 * np.sum((op.forward(x) - d) ** 2) + lam * tv_value(x, bc)
    x, _, _ = fista(op, d, lam, L, 150, 200, bc)
    xc = _cp_full_problem(op, d, lam, bc, 30000)
    assert E(x) <= E(xc) * (1 + 2e-4)
    assert np.linalg.norm(x - xc) / np.linalg.norm(xc) < 1e-2


def test_restart_and_backtracking_fire_for_too_large_step():
    """With L underestimated 20x the energy increases; restart + halving must keep E monotone."""
    op, d, L = _problem(noise=0.1)
    log = FistaLog()
    fista(op, d, 0.02, L / 20.0, 20, 30, "dirichlet", log=log)
    assert any(f > 1 for f in log.flags)                  # at least one halving happened
    e = log.energy
    # after a successful backtrack the energy is not above the previous one
    for k in range(1, len(e)):
        if 1 <= log.flags[k] <= 6:
            assert e[k] <= e[k - 1] * (1 + 1e-12) or log.flags[k] == 6


def test_bregman_residual_decreases_monotonically():
    """The data residual ||C A p^k - f|| of the Bregman iterates decreases with k (Sec. 4.5)."""
    op, d, L = _problem(noise=0.2)
    _, res = bregman(op, d, 0.2, L, 5, 40, 40, "dirichlet")
    assert all(b < a for a, b in zip(res[:-1], res[1:]))


def test_power_iteration_matches_dense_spectral_norm():
    g = Grid(8, 8, 8, dx=1e-4, c0=1500.0, dt=2e-8, nt=24, pml_size=2)
    smp = Sampling.points(64, 16, 2)
    op = DenseOperator(g, smp)
    ref = np.linalg.norm(op.M, 2) ** 2
    x0 = np.random.default_rng(1).standard_normal(g.shape)
    lam = power_iteration(op, x0, 200)
    assert abs(lam - ref) / ref < 1e-8
