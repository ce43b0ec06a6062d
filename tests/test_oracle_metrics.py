"""Pins of the oracle's thresholded PSNR (eq. PSNR), with examples worked by hand."""

import math

import numpy as np

from oracle.metrics import psnr


def test_psnr_four_voxel_example():
    # p0 = [1, 0.5, 0.05, 0]: max 1, 0.05 < 0.1 is zeroed -> [1, 0.5, 0, 0]
    # p  = [2, 0.8, 0.2, -1]: clip -> [2, 0.8, 0.2, 0], /2 -> [1, 0.4, 0.1, 0]; 0.1 >= 0.1 is kept
    # diff = [0, -0.1, 0.1, 0] -> MSE = 0.02/4 = 0.005 -> PSNR = -10 log10(0.005)
    p0 = np.array([1.0, 0.5, 0.05, 0.0])
    p = np.array([2.0, 0.8, 0.2, -1.0])
    assert abs(psnr(p, p0) - (-10 * math.log10(0.005))) < 1e-12


def test_psnr_threshold_edge_just_below():
    # 0.0999 < 0.1 is dropped: p -> [1, 0, 0, 0], p0 -> [1, 0, 0, 0] -> identical -> inf
    p = np.array([1.0, 0.0999, 0.0, 0.0])
    p0 = np.array([1.0, 0.0, 0.0, 0.0])
    assert psnr(p, p0) == float("inf")


def test_psnr_scale_invariant_and_all_zero():
    p0 = np.array([0.3, 0.6, 0.0, 0.9])
    assert psnr(5.0 * p0, p0) == float("inf")
    # an all-negative reconstruction clips to zero: MSE = mean(p0~^2) = (1/9 + 4/9 + 1)/4
    mse = (1 / 9 + 4 / 9 + 1.0) / 4
    assert abs(psnr(-p0, p0) - (-10 * math.log10(mse))) < 1e-12


def test_psnr_evaluation_region_worked_example():
    """eval_region on an 8^3 grid with P = 2: z in [1, nz - 2P) = [1, 4), y and x in [P, n - P) = [2, 6).

    N = 3 * 4 * 4 = 48 voxels. Both volumes peak at 1.0 inside the region. Large values
    planted on the sensor layer z = 0, on the first z-PML layer z = 4, deep in the z-PML
    and one cell into each lateral PML face would take over the maximum (and so every
    normalised value) if any of them were inside. Inside, p differs from p0 by 0.5 at the
    first corner (1, 2, 2) and by 0.25 at the last corner (3, 5, 5), both above the 0.1
    threshold: squared error 0.25 + 0.0625 = 0.3125, PSNR = -10 log10(0.3125 / 48).
    """
    from oracle import Grid
    from oracle.metrics import eval_region
    g = Grid(8, 8, 8, dx=1e-4, c0=1500.0, dt=2e-8, nt=2, pml_size=2)
    p0 = np.zeros((8, 8, 8))
    p0[2, 3, 3] = 1.0
    p0[0, 4, 4] = 9.0                     # sensor layer
    p0[5, 4, 4] = 9.0                     # z-PML
    p = p0.copy()
    p[0, 4, 4] = 0.0
    p[5, 4, 4] = 0.0
    p[0, 3, 3] = 50.0                     # z = 0
    p[4, 3, 3] = 40.0                     # z = nz - 2P, first PML layer
    p[7, 3, 3] = 30.0
    p[2, 1, 3] = p[2, 6, 3] = p[2, 3, 1] = p[2, 3, 6] = 20.0   # y, x = P - 1 and n - P
    p[1, 2, 2] = 0.5                      # first corner of the region
    p[3, 5, 5] = 0.25                     # last corner of the region
    reg = eval_region(g)
    assert p0[reg].size == 48
    assert abs(psnr(p, p0, reg) - (-10 * math.log10(0.3125 / 48))) < 1e-12
