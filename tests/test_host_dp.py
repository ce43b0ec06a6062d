"""Host logic of the library's discrepancy-principle search (paper_1605_00133_amd.dp)
on functions with a known root (no GPU): the same bar as the oracle's search."""

import math

import pytest

from paper_1605_00133_amd.dp import bregman_stop, discrepancy_search


@pytest.mark.parametrize("lo,hi", [(0.1, 2.0), (3.0, 5.0), (1e-4, 1e-3)])
def test_search_finds_the_known_root(lo, hi):
    lam0, kappa, tol = 2.0, 1.25, 0.01
    lam, d, hist = discrepancy_search(lambda l: 1.0 + (l / lam0) ** 2, lo, hi, kappa, tol)
    assert abs(d - kappa) <= tol
    assert abs(lam - 0.5 * lam0) <= 1.1 * tol * lam0
    assert len(hist) >= 2


def test_search_rejects_a_flat_discrepancy():
    with pytest.raises(ValueError):
        discrepancy_search(lambda l: 1.0, 0.1, 1.0, max_grow=3)


def test_bregman_stop():
    n, sigma = 100, 0.5
    s = math.sqrt(n) * sigma
    assert bregman_stop([3.0 * s, 1.5 * s, 1.2 * s, 1.1 * s], n, sigma) == 3
    assert bregman_stop([3.0 * s], n, sigma) is None
