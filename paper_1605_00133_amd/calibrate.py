"""Regularisation-parameter choice by the discrepancy principle (eq. DiscPr).

The paper selects lambda so that the data misfit of the TV+ solution explains
the data no more than up to the noise level: ||C A p_lambda - f|| / (sqrt(M) sigma)
= kappa with kappa = 1.25, found by an interval search that linearly
interpolates the discrepancy inside the current interval, stopped at a
tolerance of 0.01 (Sec. 5.2). The Bregman iteration then starts from
lambda_Br = 10 lambda_TV+. Reading: M counts every entry of f (M_c M_t), since
the printed denominator sqrt(M_c) sigma ignores the time samples.

Host-side driver only: every evaluation is a pat_reconstruct call on the GPU.
"""

import math

import numpy as np


def discrepancy(plan, f, p, lam, L, sigma, n_inner, n_prox, bc="dirichlet"):
    from . import pat as P
    out = P.pat_reconstruct(plan, f, p, lam, L, n_outer=1, n_inner=n_inner, n_prox=n_prox, bc=bc,
                            restart=True)
    m = plan.grid.nt * plan.mc
    return float(out["residual"][-1]) / (math.sqrt(m) * sigma)


def dp_search(plan, f, p, L, sigma, lam0, n_inner=50, n_prox=50, kappa=1.25, tol=0.01, max_eval=16,
              bc="dirichlet", log=None):
    """Returns (lambda, discrepancy, evaluations) with |discrepancy - kappa| <= tol when found."""
    evals = []

    def d(lam):
        v = discrepancy(plan, f, p, lam, L, sigma, n_inner, n_prox, bc)
        evals.append((lam, v))
        if log:
            log(f"DP: lambda={lam:.4e} discrepancy={v:.4f}")
        return v

    lo, hi = lam0, lam0
    dlo = dhi = d(lam0)
    if abs(dlo - kappa) <= tol:
        return lam0, dlo, evals
    # bracket kappa geometrically (the discrepancy increases with lambda)
    while dlo > kappa and len(evals) < max_eval:
        hi, dhi = lo, dlo
        lo = lo / 4.0
        dlo = d(lo)
    while dhi < kappa and len(evals) < max_eval:
        lo, dlo = hi, dhi
        hi = hi * 4.0
        dhi = d(hi)
    if not (dlo <= kappa <= dhi):
        lam, v = min(evals, key=lambda e: abs(e[1] - kappa))
        return lam, v, evals
    lam, v = lo, dlo
    while len(evals) < max_eval:
        lam = lo + (kappa - dlo) * (hi - lo) / max(dhi - dlo, 1e-300)
        v = d(lam)
        if abs(v - kappa) <= tol:
            break
        if v < kappa:
            lo, dlo = lam, v
        else:
            hi, dhi = lam, v
    return lam, v, evals


def bregman_lambda(lam_tv):
    """lambda for the Bregman iteration from the TV+ one (Sec. 5.2)."""
    return 10.0 * lam_tv


__all__ = ["discrepancy", "dp_search", "bregman_lambda", "np"]
