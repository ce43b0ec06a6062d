"""GPU parity of the learned update's U-Net layers and network against the FP64 oracle.

* pooling, upsampling (and their adjoints), add + ReLU, axpby and the squared-error
  loss and gradient: against oracle/conv.py and plain formulas, to FP32 rounding
  (the loss: FP64 sum of the squared FP32 differences, 1e-12 relative);
* the 3-level U-Net (oracle/unet.py: torch FP64 on the CPU, gradients by automatic
  differentiation): the GPU multiplies BF16-rounded operands in every convolution,
  so the output is compared at that precision (relative L2 below 2e-2) and the
  hand-written backward by the gradient of every parameter tensor (relative L2
  below 8e-2, cosine above 0.996); a wrong index, sign or missing skip path
  gives errors of order one;
* the learned iteration's fallback: a model whose output layer is scaled up
  (garbage corrections) must be replaced by the plain TV+Br reconstruction.
"""

import numpy as np
import pytest

from gpu_cases import to_dev, to_host

pytestmark = pytest.mark.gpu


def _rng(s):
    return np.random.default_rng(s)


def test_resampling_and_elementwise_layers_match_oracle():
    import torch
    from oracle.conv import pool2, pool2_backward, upsample2, upsample2_backward
    from paper_1605_00133_amd import nn
    x = _rng(1).standard_normal((2, 3, 6, 10, 18))
    c = _rng(2).standard_normal((2, 3, 3, 5, 9))
    tx, tc = to_dev(x), to_dev(c)
    x32, c32 = x.astype(np.float32).astype(np.float64), c.astype(np.float32).astype(np.float64)
    assert np.allclose(to_host(nn.pool2(tx)), pool2(x32), rtol=1e-6, atol=1e-6)
    assert np.allclose(to_host(nn.pool2_backward(tc)), pool2_backward(c32), rtol=1e-7, atol=0)
    assert np.array_equal(to_host(nn.upsample2(tc)), upsample2(c32))
    assert np.allclose(to_host(nn.upsample2_backward(tx)), upsample2_backward(x32), rtol=1e-6, atol=1e-5)
    a, b = _rng(3).standard_normal(1000), _rng(4).standard_normal(1000)
    ta, tb = to_dev(a), to_dev(b)
    a32, b32 = a.astype(np.float32).astype(np.float64), b.astype(np.float32).astype(np.float64)
    assert np.allclose(to_host(nn.add_act(ta, tb, relu=True)), np.maximum(a32 + b32, 0), rtol=1e-7, atol=1e-7)
    assert np.allclose(to_host(nn.axpby(ta, tb, 0.5, -2.0, clamp0=True)), np.maximum(0.5 * a32 - 2 * b32, 0),
                       rtol=1e-6, atol=1e-6)
    g = torch.empty_like(ta)
    loss = float(nn.mse(ta, tb, grad=g, mask0=True))
    d = (a.astype(np.float32) - b.astype(np.float32)).astype(np.float64)    # the kernel subtracts in FP32
    assert abs(loss - np.mean(d * d)) <= 1e-12 * np.mean(d * d)
    assert np.allclose(to_host(g), np.where(a32 > 0, 2 * d / 1000, 0.0), rtol=1e-6, atol=1e-9)


def _params(widths, seed):
    from oracle.unet import layer_channels
    r = _rng(seed)
    out = {}
    for k, (ci, co) in layer_channels(widths).items():
        out[k] = (r.standard_normal((co, ci, 3, 3, 3)) * np.sqrt(2.0 / (27 * ci)), 0.05 * r.standard_normal(co))
    return out


@pytest.mark.parametrize("widths,n", [((4, 8, 16), 16), ((16, 32, 64), 16)])
def test_unet_forward_and_backward_match_oracle(widths, n):
    import torch
    from oracle.unet import loss_and_grads
    from paper_1605_00133_amd import nn
    from paper_1605_00133_amd.unet import UNet
    prm = _params(widths, 5)
    net = UNet(widths, device="cuda:0")
    net.load_state_dict({f"{k}.{i}": torch.from_numpy(wb[i]) for k, wb in prm.items() for i in range(2)})
    r = _rng(6)
    p = np.abs(r.standard_normal((2, 1, n, n, n)))
    z = p + 0.3 * r.standard_normal((2, 1, n, n, n))
    t = np.abs(r.standard_normal((2, 1, n, n, n)))
    p, z, t = (a.astype(np.float32).astype(np.float64) for a in (p, z, t))
    loss_ref, out_ref, g_ref = loss_and_grads(prm, p, z, t)
    x = to_dev(np.concatenate([p, z], axis=1))
    o = net.forward(x, keep=True)
    out = nn.axpby(to_dev(z), o, 1.0, 1.0, clamp0=True)
    dout = torch.empty_like(out)
    loss = float(nn.mse(out, to_dev(t), grad=dout, mask0=True))
    grads = net.backward(dout)
    e_out = np.linalg.norm(to_host(out) - out_ref) / np.linalg.norm(out_ref)
    print(f"U-Net {widths} at {n}^3: output rel L2 {e_out:.2e}, loss {loss:.6e} vs {loss_ref:.6e}")
    assert e_out < 2e-2
    assert abs(loss - loss_ref) < 2e-2 * loss_ref
    for k in g_ref:
        for i in range(2):
            a, b = to_host(grads[k][i]).ravel(), g_ref[k][i].ravel()
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            cos = float(a @ b / (np.linalg.norm(a) * np.linalg.norm(b)))
            print(f"  {k}.{'wb'[i]}: rel L2 {rel:.2e}, cosine {cos:.6f}")
            assert rel < 8e-2 and cos > 0.996, (k, i, rel, cos)


def test_learned_fallback_to_plain_solver():
    """Output layer scaled by 1e4: the learned residual exceeds plain FISTA's, so the TV+Br result is returned."""
    import torch
    from paper_1605_00133_amd import pat as P
    from paper_1605_00133_amd.learned_unet import LearnedUNetRecon, make_case, make_plan, reconstruct_with_fallback
    from synthetic import gaussian_volume
    plan = make_plan(32, "hadamard")
    case = make_case(plan, 5000, "hadamard")
    L = P.pat_power_iteration(plan, to_dev(gaussian_volume(plan.vol_shape, 8)), 10)
    model = LearnedUNetRecon(2, (4, 8, 16), 0)
    for net in model.nets:
        net.params["c11"][0].mul_(1e4)
        net.params["c11"][1].fill_(3.0)
    p, info = reconstruct_with_fallback(model, plan, case["f"], L, case["lam_tv"], case["lam_br"], p_ref=case["p0"])
    print(info)
    assert info["fallback"] and info["residual_learned"] > info["residual_plain_same_pairs"]
    q = torch.empty(plan.vol_shape, dtype=torch.float32, device="cuda:0")
    P.pat_reconstruct(plan, case["f"], q, case["lam_br"], L, n_outer=5, n_inner=50, n_prox=50, bc="dirichlet")
    assert torch.equal(p, q)
