"""96^3 grids (transforms of length 96 = 12 * 8 and 48 = 12 * 4, radix-3 butterflies).

* A and A^T at 96^3 (Nt = 24, random 25 % single points) against the FP64 oracle
  computed here, line and slab schemes, within 1e-5 relative L2;
* the differentiation workload: a batch of four 96^3 volumes, Nt = 560, random 25 %
  single points, through paper_1605_00133_amd.autograd.measure (backward = the
  library's A^T C^T). The gradient of L = 1/2 sum_i ||C A p_i - b_i||^2 is checked
  against the FP64 oracle gradients stored by tests/golden/make_autograd96_fixtures.py
  (sampled z-slices incl. the sensor plane and a z-PML slice, and the norms) within
  1e-5, and against central differences along 16 random directions d (seeded
  N(0, 1) fields smoothed by a Gaussian of 2 voxels and scaled to unit RMS per
  voxel). L is quadratic, so the central difference has no truncation error at any
  eps; what limits it is the rounding of the FP32 data. An evaluation of L from data
  f = C A x with per-element errors e_i carries the error sum_i r_i e_i (r = f - b),
  of standard deviation about delta ||r o f|| when |e_i| ~ delta |f_i|; two
  evaluations divided by 2 eps give a central-difference error of about
  sqrt(2) delta ||r o f|| / (2 eps). With delta = 1e-5 (the tolerance of A) and four
  standard deviations this is the bound asserted at eps = 1e-3 (the configuration's
  step). The directions are nearly orthogonal to the gradient (|cos| ~ 1e-4-1e-3),
  so at that step the measured differences are 3e-5-2e-3 of <grad, d>; at eps = 1 the
  same noise is a thousand times smaller and the central difference must agree
  within 1e-4 (measured 3e-7-3e-6). The backward is A^T itself, so it keeps no tape
  of the 560 steps and needs no checkpoints.
"""

import os

import numpy as np
import pytest

import oracle
from oracle.sampling import apply_c, apply_ct
from gpu_cases import empty, gaussian_data, gpu_plan, oracle_grid, oracle_sampling, rel_l2, to_dev, to_host
from synthetic import vessel_phantom

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL_OP = 1e-5


@pytest.mark.parametrize("scheme", ["line", "slab"])
def test_operator_96_matches_oracle(scheme):
    from paper_1605_00133_amd import pat as P
    n, nt = 96, 24
    g = oracle_grid(n, nt)
    smp = oracle_sampling("points", n)
    p0 = vessel_phantom((n, n, n), 8, 24, 1.0, 4.0, 1)
    y = gaussian_data((nt, smp.mc), 5)
    op = oracle.WaveOperator(g)
    f_ref = apply_c(op.forward_planes(p0), smp)
    p_ref = op.adjoint_planes(apply_ct(y, smp, n, n))
    plan = gpu_plan(n, nt, smp)
    plan.set_scheme(scheme)
    f = empty(plan.data_shape)
    p = empty(plan.vol_shape)
    P.pat_forward(plan, to_dev(p0), f)
    P.pat_adjoint(plan, to_dev(y), p)
    ef, ea = rel_l2(to_host(f), f_ref), rel_l2(to_host(p), p_ref)
    print(f"96^3 {scheme}: forward {ef:.2e}, adjoint {ea:.2e}")
    assert ef < TOL_OP and ea < TOL_OP


def _fixture():
    path = os.path.join(GOLDEN, "grad96_points.npz")
    assert os.path.exists(path), f"committed fixture {path} is missing"
    return np.load(path)


def test_differentiation_96_batch4():
    import torch
    from paper_1605_00133_amd.autograd import measure
    fx = _fixture()
    n, nt, mc = 96, 560, 2304
    plan = gpu_plan(n, nt, oracle_sampling("points", n, mc))
    qs = torch.stack([to_dev(vessel_phantom((n, n, n), 8, 24, 1.0, 4.0, 20 + i)) for i in range(4)])
    with torch.no_grad():
        b = measure(plan, qs)
        for i in range(4):
            b[i] += float(fx["sigmas"][i]) * to_dev(gaussian_data((nt, mc), 40 + i))
    p = torch.stack([to_dev(vessel_phantom((n, n, n), 8, 24, 1.0, 4.0, 30 + i)) for i in range(4)])
    x = p.clone().requires_grad_(True)
    loss = 0.5 * ((measure(plan, x) - b).double() ** 2).sum()
    loss.backward()
    grad = x.grad.detach()
    gh = to_host(grad)
    for i in range(4):
        e = rel_l2(gh[i][fx["zs"]], fx["values"][i])
        en = abs(np.linalg.norm(gh[i]) - float(fx["norms"][i])) / float(fx["norms"][i])
        print(f"sample {i}: gradient rel L2 over z-slices {list(fx['zs'])} {e:.2e}, |grad| rel diff {en:.2e}")
        assert e < TOL_OP and en < TOL_OP

    def L(v):
        with torch.no_grad():
            return 0.5 * float(((measure(plan, v) - b).double() ** 2).sum())

    with torch.no_grad():
        f = measure(plan, p).double()
        rf = float(((f - b.double()) * f).norm())
    delta = TOL_OP
    from scipy.ndimage import gaussian_filter
    worst = {1e-3: 0.0, 1.0: 0.0}
    for k in range(16):
        dh = np.stack([gaussian_filter(gaussian_data((n, n, n), 100 + 4 * k + i), 2.0) for i in range(4)])
        d = to_dev(dh / np.sqrt(np.mean(dh * dh)))
        an = float((grad.double() * d.double()).sum())
        for eps in (1e-3, 1.0):
            fd = (L(p + eps * d) - L(p - eps * d)) / (2 * eps)
            bound = 4.0 * np.sqrt(2.0) * delta * rf / (2 * eps)
            worst[eps] = max(worst[eps], abs(fd - an) / abs(an))
            print(f"direction {k}, eps {eps:g}: central difference {fd:.8e}, autograd {an:.8e}, "
                  f"difference {abs(fd - an):.2e} (noise bound {bound:.2e})")
            if eps == 1.0:
                assert abs(fd - an) <= 1e-4 * abs(an)
            else:
                assert abs(fd - an) <= bound
    print(f"||r o f|| = {rf:.4e}; worst relative difference over 16 directions: eps 1e-3 {worst[1e-3]:.2e}, "
          f"eps 1 {worst[1.0]:.2e}")
