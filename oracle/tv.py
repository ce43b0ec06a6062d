"""Discrete isotropic total variation and the positivity-constrained TV prox.

Oracle module: test infrastructure only, never called by the GPU path.

TV (App. A): the sum over voxels of the Euclidean norm of the forward
differences in x, y and z. With Neumann boundaries the difference past the
last voxel of a line is zero. With Dirichlet boundaries the jumps to zero at
the faces are added; this is written out as the Neumann TV of the volume
zero-padded by one voxel on every face (pad voxels held at 0).

Prox (eq. Prox with J = TV + indicator{p >= 0}, App. B): a positivity-
constrained TV denoising problem, solved by the primal-dual hybrid gradient
method of Chambolle and Pock (accelerated variant, their Algorithm 2, with the
1-strongly convex data term), as the paper states:

    q = max(0, v); y = y0 (or 0); qbar = q; tau = sigma = 1/sqrt(12)
    repeat n_iter times:
        y    <- y + sigma grad(qbar);  y_i <- y_i / max(1, |y_i| / alpha)
        qn   <- max(0, (q + tau div(y) + tau v) / (1 + tau))      (pad := 0)
        theta = 1/sqrt(1 + 2 tau); tau <- theta tau; sigma <- sigma / theta
        qbar <- qn + theta (qn - q);  q <- qn

||grad||^2 <= 12 in 3D, so tau*sigma*||grad||^2 <= 1 holds from the start.
"""

import numpy as np


def _pad(p):
    return np.pad(p, 1)


def _unpad(p):
    return p[1:-1, 1:-1, 1:-1]


def grad(p):
    """Forward differences with Neumann ends -> (3, *shape), components (x, y, z)."""
    gx = np.zeros_like(p)
    gy = np.zeros_like(p)
    gz = np.zeros_like(p)
    gx[:, :, :-1] = p[:, :, 1:] - p[:, :, :-1]
    gy[:, :-1, :] = p[:, 1:, :] - p[:, :-1, :]
    gz[:-1, :, :] = p[1:, :, :] - p[:-1, :, :]
    return np.stack([gx, gy, gz])


def div(y):
    """Negative adjoint of grad: <grad p, y> = -<p, div y>."""
    yx, yy, yz = y
    d = np.zeros_like(yx)
    # x component: contributions -y[i] at i, +y[i-1] at i, last-index y unused
    d[:, :, :-1] += yx[:, :, :-1]
    d[:, :, 1:] -= yx[:, :, :-1]
    d[:, :-1, :] += yy[:, :-1, :]
    d[:, 1:, :] -= yy[:, :-1, :]
    d[:-1, :, :] += yz[:-1, :, :]
    d[1:, :, :] -= yz[:-1, :, :]
    return d


def _grad_bc(p, bc):
    return grad(_pad(p)) if bc == "dirichlet" else grad(p)


def tv_value(p, bc="neumann"):
    g = _grad_bc(np.asarray(p, dtype=np.float64), bc)
    return float(np.sqrt((g * g).sum(axis=0)).sum())


def dual_shape(shape, bc):
    if bc == "dirichlet":
        return (3,) + tuple(s + 2 for s in shape)
    return (3,) + tuple(shape)


def prox_tv_pos(v, alpha, n_iter, bc="neumann", dual=None):
    """argmin_{q >= 0} 1/2 ||q - v||^2 + alpha TV(q), by n_iter PDHG steps.

    Returns (q, dual). `dual` warm-starts the dual variable (shape dual_shape).
    """
    v = np.asarray(v, dtype=np.float64)
    dirichlet = bc == "dirichlet"
    vv = _pad(v) if dirichlet else v
    y = np.zeros(dual_shape(v.shape, bc)) if dual is None else np.array(dual, dtype=np.float64)
    q = np.maximum(0.0, vv)
    qbar = q.copy()
    tau = sigma = 1.0 / np.sqrt(12.0)
    for _ in range(n_iter):
        y = y + sigma * grad(qbar)
        if alpha > 0:
            nrm = np.sqrt((y * y).sum(axis=0))
            y = y / np.maximum(1.0, nrm / alpha)
        else:
            y = np.zeros_like(y)
        qn = np.maximum(0.0, (q + tau * div(y) + tau * vv) / (1.0 + tau))
        if dirichlet:
            qn = _pad(_unpad(qn))          # pad voxels stay at zero
        theta = 1.0 / np.sqrt(1.0 + 2.0 * tau)
        tau = theta * tau
        sigma = sigma / theta
        qbar = qn + theta * (qn - q)
        q = qn
    return (_unpad(q) if dirichlet else q), y
