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
