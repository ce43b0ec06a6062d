"""Regularisation parameter by the discrepancy principle (Sec. 5.2, eq. DiscPr).

The discrepancy of p_lam is ||C A p_lam - f|| / (sqrt(M_c M_t) sigma), the
residual norm being the FP64 reduction that pat_reconstruct logs for its last
iterate. The principle picks lam where the discrepancy, increasing in lam,
equals kappa (the paper: 1.25 within 0.01). The search interpolates the
discrepancy linearly in lam between the ends of a bracketing interval (regula
falsi), after widening a given interval until it brackets kappa. Bregman
iterations (started at 10 lam) stop at the first outer step whose logged
discrepancy is below kappa. Every reconstruction runs in the library; this
module is control flow on scalars.
"""

import math

from . import pat as P


def _regula_falsi(disc, lo, hi, kappa, tol, max_iter, grow, max_grow):
    seen = []

    def at(lam):
        seen.append((lam, float(disc(lam))))
        return seen[-1][1]

    dl, dh = at(lo), at(hi)
    k = 0
    while dl >= kappa and k < max_grow:   # widen downwards
        lo, k = lo / grow, k + 1
        dl = at(lo)
    k = 0
    while dh <= kappa and k < max_grow:   # widen upwards
        hi, k = hi * grow, k + 1
        dh = at(hi)
    if not (dl < kappa < dh):
        raise ValueError(f"no interval brackets kappa = {kappa} (discrepancy {dl:.3g} .. {dh:.3g})")
    best = min(((lo, dl), (hi, dh)), key=lambda t: abs(t[1] - kappa))
    for _ in range(max_iter):
        if abs(best[1] - kappa) <= tol:
            break
        lam = lo + (hi - lo) * (kappa - dl) / (dh - dl)
        d = at(lam)
        best = (lam, d)
        if d < kappa:
            lo, dl = lam, d
        else:
            hi, dh = lam, d
    return best[0], best[1], seen


def discrepancy_search(disc, lam_lo, lam_hi, kappa=1.25, tol=0.01, max_iter=30, grow=10.0, max_grow=8):
    """lam with |disc(lam) - kappa| <= tol for an increasing disc(lam); returns (lam, disc, history)."""
    return _regula_falsi(disc, float(lam_lo), float(lam_hi), kappa, tol, max_iter, grow, max_grow)


def tv_lambda(plan, f, p, sigma, L, lam_lo, lam_hi, n_inner=50, n_prox=50, bc="dirichlet", kappa=1.25, tol=0.01,
              max_iter=30):
    """The TV+ parameter by the discrepancy principle. f: data [Nt][M_c] on the
    GPU, sigma its noise level, L the Lipschitz estimate. Every evaluation runs
    pat_reconstruct (n_outer = 1, n_inner FISTA steps from zero) into p, which
    holds the reconstruction of the last evaluation. Returns (lam, discrepancy,
    history)."""
    n_data = plan.data_shape[0] * plan.data_shape[1]

    def disc(lam):
        out = P.pat_reconstruct(plan, f, p, lam, L, n_outer=1, n_inner=n_inner, n_prox=n_prox, bc=bc)
        return out["residual"][-1] / (math.sqrt(n_data) * sigma)

    return discrepancy_search(disc, lam_lo, lam_hi, kappa, tol, max_iter)


def bregman_stop(bregman_residual, n_data, sigma, kappa=1.25):
    """First outer step k (1-based) of a TV+Br log (pat_reconstruct's bregman_residual)
    with discrepancy below kappa, or None."""
    for k, r in enumerate(bregman_residual, start=1):
        if r / (math.sqrt(n_data) * sigma) < kappa:
            return k
    return None
