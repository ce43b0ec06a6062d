"""Pins of the FP64 convolution oracle (oracle/conv.py) against library
routines, brute force and identities that fix every index and sign."""

import numpy as np
import pytest
from scipy import ndimage

from oracle.conv import adam_step, bf16, conv3d, conv3d_backward_input, conv3d_backward_weight


def _rng(s):
    return np.random.default_rng(s)


def test_bf16_matches_torch_and_ties_to_even():
    torch = pytest.importorskip("torch")
    a = np.concatenate([_rng(1).standard_normal(10000).astype(np.float32) * 10.0 ** _rng(2).integers(-20, 20, 10000),
                        np.array([0.0, -0.0, 1.0, 65504.0, 3.0e38, 1e-40], dtype=np.float32)]).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(bf16(a), ref)
    one = np.float32(1.0)
    ulp = 2.0 ** -7                          # bfloat16 spacing at 1
    assert bf16(one + np.float32(ulp / 2)) == 1.0                  # tie -> even (1.0)
    assert bf16(one + np.float32(3 * ulp / 2)) == 1.0 + 2 * ulp    # tie -> even (1 + 2 ulp)
    assert bf16(one + np.float32(ulp / 2 + 2.0 ** -20)) == 1.0 + ulp


def test_single_channel_is_scipy_correlate():
    x = _rng(3).standard_normal((1, 1, 5, 6, 7))
    w = _rng(4).standard_normal((1, 1, 3, 3, 3))
    ref = ndimage.correlate(x[0, 0], w[0, 0], mode="constant", cval=0.0)
    assert np.allclose(conv3d(x, w)[0, 0], ref, rtol=0, atol=1e-12)


def test_matches_torch_conv3d_float64():
    torch = pytest.importorskip("torch")
    x = _rng(5).standard_normal((2, 3, 4, 5, 6))
    w = _rng(6).standard_normal((4, 3, 3, 3, 3))
    b = _rng(7).standard_normal(4)
    ref = torch.nn.functional.conv3d(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b), padding=1)
    assert np.allclose(conv3d(x, w, b), ref.numpy(), rtol=0, atol=1e-11)
    assert np.allclose(conv3d(x, w, b, relu=True), np.maximum(ref.numpy(), 0.0), rtol=0, atol=1e-11)


def test_brute_force_tiny():
    x = _rng(8).standard_normal((1, 2, 2, 3, 4))
    w = _rng(9).standard_normal((2, 2, 3, 3, 3))
    y = np.zeros((1, 2, 2, 3, 4))
    for o in range(2):
        for z in range(2):
            for yy in range(3):
                for xx in range(4):
                    s = 0.0
                    for i in range(2):
                        for a in range(3):
                            for b in range(3):
                                for c in range(3):
                                    zz, y2, x2 = z + a - 1, yy + b - 1, xx + c - 1
                                    if 0 <= zz < 2 and 0 <= y2 < 3 and 0 <= x2 < 4:
                                        s += w[o, i, a, b, c] * x[0, i, zz, y2, x2]
                    y[0, o, z, yy, xx] = s
    assert np.allclose(conv3d(x, w), y, rtol=0, atol=1e-12)


def test_input_gradient_is_the_adjoint():
    x = _rng(10).standard_normal((2, 3, 5, 4, 6))
    w = _rng(11).standard_normal((5, 3, 3, 3, 3))
    dy = _rng(12).standard_normal((2, 5, 5, 4, 6))
    lhs = np.vdot(conv3d(x, w), dy)
    rhs = np.vdot(x, conv3d_backward_input(dy, w))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_weight_gradient_is_the_derivative():
    # sum(dy * conv(x, w) + bias) is linear in (w, bias): its derivative along
    # (dw_dir, db_dir) is the same sum with (w, bias) replaced by the direction
    x = _rng(13).standard_normal((2, 3, 4, 5, 3))
    dy = _rng(14).standard_normal((2, 4, 4, 5, 3))
    gw, gb = conv3d_backward_weight(x, dy)
    for s in range(3):
        dw = _rng(20 + s).standard_normal((4, 3, 3, 3, 3))
        db = _rng(30 + s).standard_normal(4)
        lhs = np.vdot(gw, dw) + np.vdot(gb, db)
        rhs = np.vdot(dy, conv3d(x, dw, db))
        assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_adam_first_step_moves_by_lr_times_sign():
    # at step 1 the bias-corrected moments are g and g^2: the update is lr * g / (|g| + eps)
    g = np.array([2.0, -0.5, 1e-3])
    w, m, v = adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.1, eps=1e-12)
    assert np.allclose(w, -0.1 * np.sign(g), rtol=1e-9)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
