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
    """The data residual ||C A p^k - f|| of the Bregman iterates decreases with k (Sec. 4.6)."""
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


# A worked example of the restart / backtracking branch (App. B), small enough to
# follow by hand. lam = 0 and n_prox = 0 make the prox the plain clip max(0, .),
# so every iterate is a rational number. Problem: M = diag(1, 3, 1), d = (3, 1, -1),
# x0 = 0, L = 6 so eta = 1.8 / 6 = 0.3; gradient g(x) = M (M x - d); E(x) = 1/2 |M x - d|^2.
#   E(x0) = 1/2 (9 + 1 + 1) = 5.5
#   it 1 (y = 0, t = 1): g = (-3, -3, 1), x1 = clip(0.3 * (3, 3, -1)) = (0.9, 0.9, 0),
#        E = 1/2 (2.1^2 + 1.7^2 + 1) = 4.15 < 5.5: plain step kept; beta = 0, so y = x1
#   it 2: g(x1) = (-2.1, 5.1, 1), x2 = clip(x1 - 0.3 g) = (1.53, 0, 0) (-0.63 clipped),
#        E = 1/2 (1.47^2 + 1 + 1) = 2.08045: kept; beta = (t - 1)/t_next > 0 now
#   it 3: the extrapolated step raises E, so t <- 1 and the step is retaken FROM x2 with the
#        gradient AT x2, g(x2) = (-1.47, -3, 1):
#        j = 0, step 0.3:  (1.971, 0.9, 0),   E = 1/2 (1.029^2 + 1.7^2 + 1)  = 2.4744205 > 2.08045
#        j = 1, step 0.15: (1.7505, 0.45, 0), E = 1/2 (1.2495^2 + 0.35^2 + 1) = 1.341875125: kept, flag 2
#   it 4: t was reset, so beta = 0 and y = x3; g(x3) = (-1.2495, 1.05, 1),
#        x4 = (2.12535, 0.135, 0), E = 1/2 (0.87465^2 + 0.595^2 + 1) = 1.05951881125, flag 0
# With max_backtrack = 0 the failed j = 0 step is the one kept (flag 1, E = 2.4744205 > E(x2)),
# and it 4 starts from it with beta = 0: g = (-1.029, 5.1, 1), x4 = (2.2797, 0, 0),
# E = 1/2 (0.7203^2 + 1 + 1) = 1.259416045.
# Restarting from y, using the gradient at y, keeping t, keeping the first trial step, or
# halving eta for later iterations each changes x3 or x4 by more than 0.05.
_WORKED = {
    3: ([(0.9, 0.9, 0.0), (1.53, 0.0, 0.0), (1.7505, 0.45, 0.0), (2.12535, 0.135, 0.0)],
        [0, 0, 2, 0], [4.15, 2.08045, 1.341875125, 1.05951881125]),
    0: ([(0.9, 0.9, 0.0), (1.53, 0.0, 0.0), (1.971, 0.9, 0.0), (2.2797, 0.0, 0.0)],
        [0, 0, 1, 0], [4.15, 2.08045, 2.4744205, 1.259416045]),
}


@pytest.mark.parametrize("max_backtrack", [3, 0])
def test_restart_and_backtracking_worked_example(max_backtrack):
    op = MatOp(np.diag([1.0, 3.0, 1.0]), (1, 1, 3))
    d = np.array([3.0, 1.0, -1.0])
    xs, flags, energies = _WORKED[max_backtrack]
    for k in range(1, 5):
        log = FistaLog()
        x, r, _ = fista(op, d, 0.0, 6.0, k, 0, "neumann", restart=True, max_backtrack=max_backtrack, log=log)
        assert np.allclose(x.ravel(), xs[k - 1], rtol=0, atol=1e-14), (k, x.ravel())
        assert log.flags == flags[:k]
        assert np.allclose(log.energy, energies[:k], rtol=1e-14, atol=0)
        assert np.allclose(r, op.M @ np.asarray(xs[k - 1]) - d, atol=1e-14)
