"""Choice of the regularisation parameter by the discrepancy principle (Sec. 5.2,
eq. DiscPr).

Oracle module: test infrastructure only, never called by the GPU path.

The discrepancy of a reconstruction p_lam is ||C A p_lam - f|| / (sqrt(M_c M_t) sigma)
(the paper prints sqrt(M_c) sigma although f has M_c M_t entries: read as the
noise norm of all of them). It grows with lam; the principle picks lam where it
equals kappa >= 1 (the paper: kappa = 1.25, tolerance 0.01), found by an
interval method that interpolates the discrepancy linearly between the ends of
the current interval (regula falsi in lam). Bregman iterations started from
10 lam stop at the first outer step whose discrepancy falls below kappa.
"""

import math


def discrepancy(residual_norm, n_data, sigma):
    """||C A p - f|| / (sqrt(n_data) sigma), n_data = M_c M_t."""
    return float(residual_norm) / (math.sqrt(n_data) * sigma)


def dp_search(disc, lam_lo, lam_hi, kappa=1.25, tol=0.01, max_iter=30, grow=10.0, max_grow=8):
    """lam with |disc(lam) - kappa| <= tol, disc increasing in lam.

    The interval [lam_lo, lam_hi] is first widened (lam_lo / grow, lam_hi * grow)
    until disc(lam_lo) < kappa < disc(lam_hi); then regula falsi. Returns
    (lam, disc(lam), [(lam, disc), ...] in evaluation order)."""
    hist = []

    def ev(lam):
        d = float(disc(lam))
        hist.append((lam, d))
        return d

    lo, hi = float(lam_lo), float(lam_hi)
    d_lo, d_hi = ev(lo), ev(hi)
    for _ in range(max_grow):
        if d_lo < kappa:
            break
        lo /= grow
        d_lo = ev(lo)
    for _ in range(max_grow):
        if d_hi > kappa:
            break
        hi *= grow
        d_hi = ev(hi)
    if not d_lo < kappa < d_hi:
        raise ValueError("discrepancy principle: no interval brackets kappa")
    lam, d = (lo, d_lo) if abs(d_lo - kappa) < abs(d_hi - kappa) else (hi, d_hi)
    for _ in range(max_iter):
        if abs(d - kappa) <= tol:
            break
        lam = lo + (kappa - d_lo) * (hi - lo) / (d_hi - d_lo)
        d = ev(lam)
        if d < kappa:
            lo, d_lo = lam, d
        else:
            hi, d_hi = lam, d
    return lam, d, hist


def bregman_stop(residual_norms, n_data, sigma, kappa=1.25):
    """First outer step k (1-based) whose discrepancy ||C A p^k - f|| is below kappa, or None."""
    for k, r in enumerate(residual_norms, start=1):
        if discrepancy(r, n_data, sigma) < kappa:
            return k
    return None
