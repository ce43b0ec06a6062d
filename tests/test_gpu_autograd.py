"""Differentiation through the operator: paper_1605_00133_amd.autograd.measure.

The gradient of L(p0) = 1/2 ||C A p0 - b||^2 taken by torch autograd (backward =
pat_adjoint) is checked against the FP64 oracle gradient A^T C^T (C A p0 - b),
within 1e-5 relative L2 (the operator bar), and against central differences of
L along random directions: L is quadratic, so the central difference equals the
directional derivative up to rounding (tolerance 1e-4, the loss being summed in
FP64 from FP32 data).
"""

import numpy as np
import pytest

import oracle
from oracle.sampling import apply_c, apply_ct
from gpu_cases import gaussian_data, gpu_plan, oracle_grid, oracle_sampling, phantom, rel_l2, to_dev, to_host

TOL_OP = 1e-5


def test_measure_rejects_bad_shapes():
    torch = pytest.importorskip("torch")
    from paper_1605_00133_amd.autograd import measure
    with pytest.raises(ValueError):
        measure(None, torch.zeros(4, 4))


def _setup(n=32, nt=190, kind="points"):
    g = oracle_grid(n, nt)
    smp = oracle_sampling(kind, n)
    p0 = phantom(n)
    b = gaussian_data((nt, smp.mc), 7) * 0.05
    return g, smp, p0, b, gpu_plan(n, nt, smp)


@pytest.mark.gpu
@pytest.mark.parametrize("kind", ["points", "hadamard"])
def test_gradient_matches_oracle(kind):
    import torch
    from paper_1605_00133_amd.autograd import measure
    g, smp, p0, b, plan = _setup(kind=kind)
    n = p0.shape[0]
    x = to_dev(p0).requires_grad_(True)
    f = measure(plan, x)
    loss = 0.5 * ((f - to_dev(b)) ** 2).sum()
    loss.backward()
    op = oracle.WaveOperator(g)
    r = apply_c(op.forward_planes(p0), smp) - b
    ref = op.adjoint_planes(apply_ct(r, smp, n, n))
    err = rel_l2(to_host(x.grad), ref)
    print(f"autograd {kind} 32^3: gradient rel L2 vs FP64 oracle = {err:.3e}")
    assert err < TOL_OP


@pytest.mark.gpu
def test_gradient_central_differences():
    import torch
    from paper_1605_00133_amd.autograd import measure
    _, _, p0, b, plan = _setup()
    bd = to_dev(b)

    def loss(x):
        with torch.no_grad():
            return 0.5 * float(((measure(plan, x) - bd).double() ** 2).sum())

    x = to_dev(p0).requires_grad_(True)
    (0.5 * ((measure(plan, x) - bd) ** 2).sum()).backward()
    grad = x.grad.double()
    rng = np.random.default_rng(3)
    eps = 0.1 * float(np.linalg.norm(p0))
    for _ in range(4):
        d = rng.standard_normal(p0.shape)
        d /= np.linalg.norm(d)
        dd = to_dev(d)
        fd = (loss(to_dev(p0) + eps * dd) - loss(to_dev(p0) - eps * dd)) / (2 * eps)
        an = float((grad * dd.double()).sum())
        print(f"direction: central difference {fd:.6e}, autograd {an:.6e}")
        assert abs(fd - an) <= 1e-4 * abs(an)


@pytest.mark.gpu
def test_batch_equals_single_volumes():
    import torch
    from paper_1605_00133_amd.autograd import measure
    _, _, p0, b, plan = _setup(n=32, nt=60)
    x = torch.stack([to_dev(p0), to_dev(0.5 * p0[::-1].copy())]).requires_grad_(True)
    f = measure(plan, x)
    w = torch.randn_like(f)
    (f * w).sum().backward()
    for k in range(2):
        xk = x.detach()[k].clone().requires_grad_(True)
        fk = measure(plan, xk)
        (fk * w[k]).sum().backward()
        assert torch.equal(fk, f[k].detach())
        assert torch.equal(xk.grad, x.grad[k])
