"""Thresholded PSNR (eq. PSNR), FP64.

Oracle module: test infrastructure only, never called by the GPU path.

The paper sets negative voxels and the sensor voxels of a reconstruction to
zero, scales p and p0 by their maxima, zeroes values below 0.1 of the maximum
and reports -10 log10(||p~ - p0~||^2 / N). Reading: the N voxels evaluated are
the non-PML interior with z >= 1 (the sensor layer z = 0 excluded), the
maximum is taken over that region, and the threshold keeps values >= 0.1.
"""

import numpy as np


def eval_region(g):
    P = g.pml_size
    return (slice(1, g.nz - 2 * P), slice(P, g.ny - P), slice(P, g.nx - P))


def _normalise(p):
    p = np.maximum(np.asarray(p, dtype=np.float64), 0.0)
    m = p.max() if p.size else 0.0
    if m <= 0.0:
        return np.zeros_like(p)
    p = p / m
    return np.where(p >= 0.1, p, 0.0)


def psnr(p, p0, region=None):
    if region is not None:
        p = np.asarray(p)[region]
        p0 = np.asarray(p0)[region]
    a = _normalise(p)
    b = _normalise(p0)
    mse = float(((a - b) ** 2).sum()) / a.size
    return float("inf") if mse == 0.0 else -10.0 * np.log10(mse)
