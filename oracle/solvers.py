"""FISTA with restart/backtracking, Bregman iteration and power iteration (FP64).

Oracle module: test infrastructure only, never called by the GPU path.

Problem (eq. VarReg with J = TV + indicator{p >= 0}, eq. TV+):
    min_p  E(p) = 1/2 ||C A p - d||^2 + lam * TV(p),   p >= 0.

Solver (App. B): proximal gradient descent p <- prox_{J, eta*lam}(p - eta grad D(p))
with grad D(p) = A^T C^T (C A p - d), step eta = 1.8/L where L approximates the
Lipschitz constant of A^T C^T C A (found once by power iteration), accelerated
by FISTA; when E increases the acceleration is restarted, that iteration
becomes a plain gradient step, followed if needed by up to 5 backtracking
steps that halve the step for that iteration only (eta itself is kept).

Readings where App. B is silent:
* iterate count K is fixed (no early stop), p^0 = 0 or a warm start;
* the data-space residual of the extrapolated point is formed by linearity,
  r_y = r_x + beta (r_x - r_prev), so each iteration costs one A and one A^T;
* one PDHG dual variable is carried through every prox call in call order;
* backtracking: step j = 0 is the plain gradient step with eta, steps
  j = 1..max_backtrack use eta / 2^j; the first that does not increase E is
  kept, otherwise the last one.

Bregman (eq. BregIterA/B): b^0 = 0, p^{k+1} = argmin 1/2||CAp - (f + b^k)||^2 + lam J(p),
b^{k+1} = b^k + f - C A p^{k+1}. Each outer solve warm-starts from the previous p.
"""

from dataclasses import dataclass, field
from typing import List

import numpy as np

from .sampling import apply_c, apply_ct
from .tv import prox_tv_pos, tv_value


class MeasuredOperator:
    """x -> C W_s A x and its transpose, on top of a WaveOperator and a Sampling.

    sens: optional sensor sensitivity W_s (eq. FwdSenVar), one weight per pixel of
    the detection plane [Ny][Nx] scaling that pixel's pressure time course before
    the sub-sampling; None is the ideal sensor (W_s = I)."""

    def __init__(self, wave, smp, sens=None):
        self.wave = wave
        self.smp = smp
        g = wave.g
        self.in_shape = g.shape
        self.out_shape = (g.nt, smp.mc)
        self.sens = None if sens is None else np.asarray(sens, dtype=np.float64).reshape(g.ny, g.nx)

    def forward(self, x):
        s = self.wave.forward_planes(x)
        if self.sens is not None:
            s = s * self.sens[None]
        return apply_c(s, self.smp)

    def adjoint(self, r):
        g = self.wave.g
        s = apply_ct(r, self.smp, g.ny, g.nx)
        if self.sens is not None:
            s = s * self.sens[None]
        return self.wave.adjoint_planes(s)


@dataclass
class FistaLog:
    energy: List[float] = field(default_factory=list)
    residual: List[float] = field(default_factory=list)
    tv: List[float] = field(default_factory=list)
    flags: List[int] = field(default_factory=list)     # 0 plain, 1 + j: restart with j halvings


def _energy(r, x, lam, bc):
    tv = tv_value(x, bc)
    return 0.5 * float(np.dot(r.ravel(), r.ravel())) + lam * tv, tv


def fista(op, d, lam, L, n_iter, n_prox, bc="dirichlet", x0=None, restart=True,
          max_backtrack=5, dual=None, log=None):
    """Returns (x, r_x, dual) with r_x = C A x - d."""
    eta = 1.8 / L
    shape = op.in_shape
    x0 = np.zeros(shape) if x0 is None else np.asarray(x0, dtype=np.float64)
    r_prev = op.forward(x0) - d
    e_prev, _ = _energy(r_prev, x0, lam, bc)
    x_prev = x0.copy()
    y = x0.copy()
    r_y = r_prev.copy()
    t = 1.0
    for _ in range(n_iter):
        g = op.adjoint(r_y)
        x, dual = prox_tv_pos(y - eta * g, eta * lam, n_prox, bc, dual)
        r_x = op.forward(x) - d
        e, tv = _energy(r_x, x, lam, bc)
        flag = 0
        if restart and e > e_prev:
            t = 1.0
            g = op.adjoint(r_prev)
            for j in range(max_backtrack + 1):
                step = eta / (2.0 ** j)
                x, dual = prox_tv_pos(x_prev - step * g, step * lam, n_prox, bc, dual)
                r_x = op.forward(x) - d
                e, tv = _energy(r_x, x, lam, bc)
                flag = 1 + j
                if e <= e_prev:
                    break
        t_next = (1.0 + np.sqrt(1.0 + 4.0 * t * t)) / 2.0
        beta = (t - 1.0) / t_next
        y = x + beta * (x - x_prev)
        r_y = r_x + beta * (r_x - r_prev)
        if log is not None:
            log.energy.append(e)
            log.residual.append(float(np.linalg.norm(r_x)))
            log.tv.append(tv)
            log.flags.append(flag)
        x_prev, r_prev, e_prev, t = x, r_x, e, t_next
    return x_prev, r_prev, dual


def bregman(op, f, lam, L, n_outer, n_inner, n_prox, bc="dirichlet", restart=True,
            max_backtrack=5, log=None):
    """TV+Br: returns (p, residual norms ||C A p^k - f|| for k = 1..n_outer)."""
    f = np.asarray(f, dtype=np.float64)
    b = np.zeros_like(f)
    p = np.zeros(op.in_shape)
    dual = None
    res = []
    for _ in range(n_outer):
        p, r, dual = fista(op, f + b, lam, L, n_inner, n_prox, bc, x0=p, restart=restart,
                           max_backtrack=max_backtrack, dual=dual, log=log)
        b_old = b
        b = -r                                   # = b + (f - C A p)
        res.append(float(np.linalg.norm(r + b_old)))
    return p, res


def power_iteration(op, x0, n_iter):
    """Largest eigenvalue of A^T C^T C A by n_iter power steps from x0."""
    x = np.asarray(x0, dtype=np.float64)
    x = x / np.linalg.norm(x)
    lam = 0.0
    for _ in range(n_iter):
        w = op.adjoint(op.forward(x))
        lam = float(np.linalg.norm(w))
        x = w / lam
    return lam
