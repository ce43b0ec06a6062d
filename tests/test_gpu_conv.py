"""Parity of the BF16-MFMA convolution layers (include/pat_nn.h) with the FP64
oracle (oracle/conv.py).

The GPU rounds every product operand to bfloat16 and sums in FP32; the oracle
takes the same bfloat16-rounded operands and sums in FP64. Products of two
bfloat16 values are exact in FP32, so the two differ only by FP32 summation:
relative L2 below 1e-5 for every layer (sums of at most 27 * 16 = 432 terms,
or chunked FP32 sums of a few hundred terms added in FP64 for the weights).
Sizes are ragged against the 16 x 16 tiles and the 16 x 4 output tiles of a
block (x extent 37, y extent 7, 20 output channels, K = 27 * 3 = 81), cover
both forward kernels (packed operands with the input halo in LDS for up to 64
padded input channels, the unpacked kernel above), both weight-gradient kernels
(operands in LDS for up to 64 channels each way, gathered from global memory
above) and the shapes of the learned update network.
"""

import numpy as np
import pytest

from oracle.conv import adam_step, bf16, conv3d, conv3d_backward_input, conv3d_backward_weight

pytestmark = pytest.mark.gpu
TOL = 1e-5

CASES = [  # (batch, c_in, c_out, nz, ny, nx)
    (2, 3, 20, 5, 6, 37),
    (1, 16, 16, 16, 16, 16),
    (1, 2, 16, 32, 32, 32),
    (2, 16, 1, 8, 9, 10),
    (1, 1, 1, 1, 1, 1),
    (1, 24, 24, 6, 7, 33),
    (1, 70, 5, 4, 5, 18),      # forward on the unpacked kernel (more than 64 input channels)
    (1, 5, 70, 3, 4, 17),      # five output-channel tiles: two channel groups per tile
    (1, 64, 32, 5, 6, 20),     # 64 input channels: two output planes per block, odd nz
]


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _data(case, seed):
    nb, ci, co, nz, ny, nx = case
    r = np.random.default_rng(seed)
    x = r.standard_normal((nb, ci, nz, ny, nx)).astype(np.float32)
    w = (r.standard_normal((co, ci, 3, 3, 3)) / np.sqrt(27 * ci)).astype(np.float32)
    b = r.standard_normal(co).astype(np.float32)
    dy = r.standard_normal((nb, co, nz, ny, nx)).astype(np.float32)
    return x, w, b, dy


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _host(t):
    import torch
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


@pytest.mark.parametrize("case", CASES)
def test_forward_backward_layers_match_oracle(case):
    from paper_1605_00133_amd import nn
    x, w, b, dy = _data(case, 1)
    for relu in (False, True):
        y = _host(nn.conv3d_forward(_dev(x), _dev(w), _dev(b), relu=relu))
        ref = conv3d(bf16(x), bf16(w), b.astype(np.float64), relu=relu)
        err = _rel(y, ref)
        print(f"{case} forward relu={relu}: rel L2 {err:.2e}")
        assert err < TOL
    dx = _host(nn.conv3d_backward_input(_dev(dy), _dev(w)))
    err = _rel(dx, conv3d_backward_input(bf16(dy), bf16(w)))
    print(f"{case} input grad: rel L2 {err:.2e}")
    assert err < TOL
    dw, db = nn.conv3d_backward_weight(_dev(x), _dev(dy))
    rw, rb = conv3d_backward_weight(bf16(x), bf16(dy))
    ew, eb = _rel(_host(dw), rw), _rel(_host(db), rb)
    print(f"{case} weight grad: rel L2 {ew:.2e}, bias grad {eb:.2e}")
    assert ew < TOL and eb < TOL


def test_weight_gradient_is_deterministic_and_batch_zero():
    from paper_1605_00133_amd import nn
    import torch
    x, w, b, dy = _data(CASES[0], 2)
    a = nn.conv3d_backward_weight(_dev(x), _dev(dy))
    c = nn.conv3d_backward_weight(_dev(x), _dev(dy))
    assert torch.equal(a[0], c[0]) and torch.equal(a[1], c[1])
    e = torch.empty((0, 3, 5, 6, 37), device="cuda")
    dw, db = nn.conv3d_backward_weight(e, torch.empty((0, 20, 5, 6, 37), device="cuda"))
    assert not dw.any() and not db.any()
    assert nn.conv3d_forward(e, _dev(w)).shape == (0, 20, 5, 6, 37)


def test_relu_backward_and_adam():
    from paper_1605_00133_amd import nn
    r = np.random.default_rng(3)
    y = np.maximum(r.standard_normal(100003), 0).astype(np.float32)
    g = r.standard_normal(100003).astype(np.float32)
    gd = _dev(g)
    nn.relu_backward_(_dev(y), gd)
    assert np.array_equal(_host(gd), np.where(y > 0, g, 0).astype(np.float64))
    w0, m0, v0 = (r.standard_normal(5001).astype(np.float32) for _ in range(3))
    v0 = np.abs(v0)
    wd, md, vd = _dev(w0), _dev(m0), _dev(v0)
    nn.adam_step_(wd, _dev(g[:5001]), md, vd, step=3, lr=1e-2)
    rw, rm, rv = adam_step(w0.astype(np.float64), g[:5001].astype(np.float64), m0.astype(np.float64),
                           v0.astype(np.float64), 3, lr=1e-2)
    assert _rel(_host(wd), rw) < 1e-6 and _rel(_host(md), rm) < 1e-6 and _rel(_host(vd), rv) < 1e-6


def test_autograd_equals_layer_calls_and_oracle_chain():
    import torch
    from paper_1605_00133_amd import nn
    x, w1, b1, _ = _data((1, 2, 16, 12, 12, 20), 4)
    _, w2, b2, t = _data((1, 16, 1, 12, 12, 20), 5)
    xd = _dev(x).requires_grad_(True)
    p = [_dev(a).requires_grad_(True) for a in (w1, b1, w2, b2)]
    h = nn.conv3d(xd, p[0], p[1], relu=True)
    y = nn.conv3d(h, p[2], p[3])
    (y * _dev(t)).sum().backward()
    # the same gradients by explicit layer calls
    with torch.no_grad():
        g2w, g2b = nn.conv3d_backward_weight(h.detach(), _dev(t))
        gh = nn.conv3d_backward_input(_dev(t), p[2].detach())
        nn.relu_backward_(h.detach(), gh)
        g1w, g1b = nn.conv3d_backward_weight(xd.detach(), gh)
        gx = nn.conv3d_backward_input(gh, p[0].detach())
    for got, ref in ((p[2].grad, g2w), (p[3].grad, g2b), (p[0].grad, g1w), (p[1].grad, g1b), (xd.grad, gx)):
        assert torch.equal(got, ref)
    # against the FP64 chain with the same bfloat16 rounding points: the FP32 and
    # FP64 intermediates can round to neighbouring bfloat16 values (2^-8 apart)
    # where they straddle a rounding boundary, hence 1e-3 here
    ho = conv3d(bf16(x), bf16(w1), b1.astype(np.float64), relu=True)
    yo = conv3d(bf16(ho), bf16(w2), b2.astype(np.float64))
    assert _rel(_host(y.detach()), yo) < 1e-3
    gho = conv3d_backward_input(bf16(t), bf16(w2)) * (ho > 0)
    assert _rel(_host(p[0].grad), conv3d_backward_weight(bf16(x), bf16(gho))[0]) < 1e-3
