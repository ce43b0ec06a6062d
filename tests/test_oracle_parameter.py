"""Pins of the discrepancy-principle search (oracle.parameter) on functions with
a known root, independent of the operator: d(lam) = 1 + (lam/lam0)^2 has
d = kappa at lam0 sqrt(kappa - 1); the search must land within the tolerance."""

import math

import pytest

from oracle.parameter import bregman_stop, discrepancy, dp_search


def test_discrepancy_is_residual_over_noise_norm():
    n, sigma = 740 * 2048, 0.03
    assert discrepancy(1.3 * math.sqrt(n) * sigma, n, sigma) == pytest.approx(1.3, rel=1e-14)


@pytest.mark.parametrize("lo,hi", [(0.1, 2.0), (3.0, 5.0), (1e-4, 1e-3)])
def test_dp_search_finds_the_known_root(lo, hi):
    lam0, kappa, tol = 2.0, 1.25, 0.01
    lam, d, hist = dp_search(lambda l: 1.0 + (l / lam0) ** 2, lo, hi, kappa, tol)
    assert abs(d - kappa) <= tol
    # d'(lam*) = 2 lam* / lam0^2 = 1 / lam0 at lam* = lam0 / 2: |lam - lam*| <= tol lam0 (+ curvature)
    assert abs(lam - 0.5 * lam0) <= 1.1 * tol * lam0
    assert all(abs(h[1] - (1.0 + (h[0] / lam0) ** 2)) < 1e-15 for h in hist)


def test_dp_search_rejects_a_flat_discrepancy():
    with pytest.raises(ValueError):
        dp_search(lambda l: 1.0, 0.1, 1.0, 1.25, 0.01, max_grow=3)


def test_bregman_stop_is_the_first_step_below_kappa():
    n, sigma = 100, 0.5
    s = math.sqrt(n) * sigma
    assert bregman_stop([3.0 * s, 1.5 * s, 1.2 * s, 1.1 * s], n, sigma, 1.25) == 3
    assert bregman_stop([3.0 * s, 2.0 * s], n, sigma, 1.25) is None
