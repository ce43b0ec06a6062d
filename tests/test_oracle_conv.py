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


def test_pool2_and_upsample2_brute_force_and_adjoints():
    from oracle.conv import pool2, pool2_backward, upsample2, upsample2_backward
    x = _rng(20).standard_normal((2, 3, 4, 6, 8))
    ref = np.zeros((2, 3, 2, 3, 4))
    for i in np.ndindex(ref.shape):
        b, c, z, y, w = i
        ref[i] = x[b, c, 2 * z:2 * z + 2, 2 * y:2 * y + 2, 2 * w:2 * w + 2].mean()
    assert np.allclose(pool2(x), ref, rtol=0, atol=1e-15)
    u = upsample2(ref)
    for i in np.ndindex(u.shape):
        b, c, z, y, w = i
        assert u[i] == ref[b, c, z // 2, y // 2, w // 2]
    assert np.allclose(pool2(upsample2(ref)), ref, rtol=0, atol=1e-15)   # pooling undoes upsampling
    yc = _rng(21).standard_normal(ref.shape)
    yf = _rng(22).standard_normal(x.shape)
    assert abs(np.vdot(pool2(x), yc) - np.vdot(x, pool2_backward(yc))) < 1e-12
    assert abs(np.vdot(upsample2(yc), yf) - np.vdot(yc, upsample2_backward(yf))) < 1e-12


def _small_unet(widths=(2, 3, 4), seed=30):
    from oracle.unet import layer_channels
    r = _rng(seed)
    return {k: (0.15 * r.standard_normal((co, ci, 3, 3, 3)), 0.1 * r.standard_normal(co))
            for k, (ci, co) in layer_channels(widths).items()}


def test_unet_oracle_forward_is_the_composition_of_the_layer_oracle():
    """The torch U-Net (avg_pool3d, nearest interpolate, conv3d) against the plain layer oracle."""
    pytest.importorskip("torch")
    import torch
    from oracle.conv import pool2, upsample2
    from oracle.unet import net
    prm = _small_unet()
    x = _rng(31).standard_normal((2, 2, 8, 8, 8))
    c = lambda t, k, relu=True: conv3d(t, prm[k][0], prm[k][1], relu=relu)
    a2 = c(c(x, "c1"), "c2")
    a4 = c(c(pool2(a2), "c3"), "c4")
    a6 = c(c(pool2(a4), "c5"), "c6")
    a7 = np.maximum(c(upsample2(a6), "c7", False) + a4, 0)
    a8 = c(a7, "c8")
    a9 = np.maximum(c(upsample2(a8), "c9", False) + a2, 0)
    ref = c(c(a9, "c10"), "c11", False)
    tp = {k: (torch.from_numpy(w), torch.from_numpy(b)) for k, (w, b) in prm.items()}
    got = net(tp, torch.from_numpy(x)).numpy()
    assert np.abs(ref).max() > 0.1
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_unet_oracle_gradients_match_central_differences():
    pytest.importorskip("torch")
    from oracle.unet import loss_and_grads
    prm = _small_unet(seed=32)
    r = _rng(33)
    p = np.abs(r.standard_normal((1, 1, 8, 8, 8)))
    z = r.standard_normal((1, 1, 8, 8, 8)) + 1.0
    t = np.abs(r.standard_normal((1, 1, 8, 8, 8)))
    _, _, g = loss_and_grads(prm, p, z, t)
    eps = 1e-6
    for name, idx in [("c1", (0, 1, 2, 1, 0)), ("c6", (3, 2, 1, 1, 1)), ("c9", (1, 2, 0, 2, 2)), ("c11", (0, 0, 1, 1, 1))]:
        w = prm[name][0]
        old = w[idx]
        w[idx] = old + eps
        lp, _, _ = loss_and_grads(prm, p, z, t)
        w[idx] = old - eps
        lm, _, _ = loss_and_grads(prm, p, z, t)
        w[idx] = old
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[name][0][idx]) <= 1e-6 * max(1.0, abs(fd)), (name, fd, g[name][0][idx])
    bfd = []
    b = prm["c7"][1]
    b[1] += eps
    lp, _, _ = loss_and_grads(prm, p, z, t)
    b[1] -= 2 * eps
    lm, _, _ = loss_and_grads(prm, p, z, t)
    b[1] += eps
    bfd = (lp - lm) / (2 * eps)
    assert abs(bfd - g["c7"][1][1]) <= 1e-6 * max(1.0, abs(bfd))
