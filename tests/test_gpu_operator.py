"""GPU (gfx950) parity of A, A^T and C against the FP64 oracle, through the C ABI.

Tolerances (stated per result): A and A^T within 1e-5 relative L2 of FP64;
index arrays bit-exact; the sampling operators alone within FP32 rounding.
"""

import numpy as np
import pytest

import oracle
from oracle.sampling import apply_c, apply_ct
from gpu_cases import (empty, gaussian_data, gaussian_volume, gpu_plan, oracle_grid, oracle_sampling, phantom,
                       rel_l2, to_dev, to_host)

pytestmark = pytest.mark.gpu

TOL_OP = 1e-5


def _fwd_case(n, nt, kind, pml=8, x=None, bits=64, scheme="line"):
    g = oracle_grid(n, nt, pml)
    smp = oracle_sampling(kind, n)
    x = phantom(n, pml) if x is None else x
    ref = apply_c(oracle.WaveOperator(g).forward_planes(x), smp)
    from paper_1605_00133_amd import pat as P
    plan = gpu_plan(n, nt, smp, pml)
    plan.set_fft_precision(bits)
    plan.set_scheme(scheme)
    f = empty(plan.data_shape)
    P.pat_forward(plan, to_dev(x), f)
    return to_host(f), ref


def _adj_case(n, nt, kind, pml=8, seed=5, bits=64, scheme="line"):
    g = oracle_grid(n, nt, pml)
    smp = oracle_sampling(kind, n)
    y = gaussian_data((nt, smp.mc), seed)
    ref = oracle.WaveOperator(g).adjoint_planes(apply_ct(y, smp, n, n))
    from paper_1605_00133_amd import pat as P
    plan = gpu_plan(n, nt, smp, pml)
    plan.set_fft_precision(bits)
    plan.set_scheme(scheme)
    p = empty(plan.vol_shape)
    P.pat_adjoint(plan, to_dev(y), p)
    return to_host(p), ref


CASES = [(16, 40, "full", 4), (32, 190, "points", 8), (32, 190, "hadamard", 8), (32, 190, "full", 8),
         (64, 24, "points", 8)]


@pytest.mark.parametrize("scheme", ["line", "slab"])
@pytest.mark.parametrize("n,nt,kind,pml", CASES)
def test_forward_matches_oracle(n, nt, kind, pml, scheme):
    got, ref = _fwd_case(n, nt, kind, pml, scheme=scheme)
    err = rel_l2(got, ref)
    print(f"forward {n}^3 nt={nt} {kind} {scheme}: rel L2 vs FP64 = {err:.3e}")
    assert err < TOL_OP


@pytest.mark.parametrize("scheme", ["line", "slab"])
@pytest.mark.parametrize("n,nt,kind,pml", CASES)
def test_adjoint_matches_oracle(n, nt, kind, pml, scheme):
    got, ref = _adj_case(n, nt, kind, pml, scheme=scheme)
    err = rel_l2(got, ref)
    print(f"adjoint {n}^3 nt={nt} {kind} {scheme}: rel L2 vs FP64 = {err:.3e}")
    assert err < TOL_OP


def _special_volume(n, seed):
    """A volume made only of what the line layout treats apart: fields constant
    or alternating along x or y or z (spectra on the planes kx, ky or kz = 0 or
    N/2, where only one line of each conjugate pair is stored), among them the
    four real z lines kx, ky in {0, N/2} that share two slots."""
    rng = np.random.default_rng(seed)
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    v = np.zeros((n, n, n))
    for ax in (0, 1):
        for ay in (0, 1):
            v += (-1.0) ** (ax * x + ay * y) * rng.standard_normal(n)[z]
    for a in (0, 1):
        v += (-1.0) ** (a * z) * rng.standard_normal((n, n))[y, x]
        v += (-1.0) ** (a * x) * rng.standard_normal((n, n))[z, y]
        v += (-1.0) ** (a * y) * rng.standard_normal((n, n))[z, x]
    return v


@pytest.mark.parametrize("n,nt,pml", [(16, 40, 4), (32, 60, 8)])
def test_line_layout_special_planes(n, nt, pml):
    """Forward of a volume, and adjoint of data, that live only on the
    self-conjugate planes and real lines (full sampling): line scheme vs FP64."""
    got, ref = _fwd_case(n, nt, "full", pml, x=_special_volume(n, 11))
    e1 = rel_l2(got, ref)
    rng = np.random.default_rng(12)
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    y = sum((-1.0) ** (ax * xx + ay * yy)[None] * rng.standard_normal(nt)[:, None, None]
            for ax in (0, 1) for ay in (0, 1)).reshape(nt, n * n)
    g = oracle_grid(n, nt, pml)
    smp = oracle_sampling("full", n)
    ref = oracle.WaveOperator(g).adjoint_planes(apply_ct(y, smp, n, n))
    from paper_1605_00133_amd import pat as P
    plan = gpu_plan(n, nt, smp, pml)
    p = empty(plan.vol_shape)
    P.pat_adjoint(plan, to_dev(y), p)
    e2 = rel_l2(to_host(p), ref)
    print(f"special planes {n}^3 nt={nt}: forward {e1:.3e}, adjoint {e2:.3e}")
    assert e1 < TOL_OP and e2 < TOL_OP


@pytest.mark.parametrize("kind", ["points", "hadamard"])
def test_fp32_butterfly_variant(kind):
    """The FP32-arithmetic variant of the propagator (pat_plan_set_fft_precision(32)) at 32^3."""
    got, ref = _fwd_case(32, 190, kind, bits=32)
    e1 = rel_l2(got, ref)
    got, ref = _adj_case(32, 190, kind, bits=32)
    e2 = rel_l2(got, ref)
    print(f"FP32 butterflies 32^3 {kind}: forward {e1:.3e}, adjoint {e2:.3e}")
    assert e1 < TOL_OP and e2 < TOL_OP


@pytest.mark.parametrize("scheme", ["line", "slab"])
def test_forward_without_pml_closed_form_random_input(scheme):
    """P = 0 and white-noise p0 excite every mode including the Nyquist planes."""
    n, nt = 32, 60
    x = gaussian_volume((n, n, n), 3)
    got, ref = _fwd_case(n, nt, "full", pml=0, x=x, scheme=scheme)
    err = rel_l2(got, ref)
    print(f"forward 32^3 no PML white noise: rel L2 = {err:.3e}")
    assert err < TOL_OP


@pytest.mark.parametrize("scheme", ["line", "slab"])
@pytest.mark.parametrize("nt", [1, 2, 3])
def test_short_series_edge_cases(nt, scheme):
    """Nt = 1 (no time step: plane of p0 only), 2 and 3, with a volume that is nonzero on the plane."""
    x = gaussian_volume((32, 32, 32), 13)
    got, ref = _fwd_case(32, nt, "points", x=x, scheme=scheme)
    e1 = rel_l2(got, ref)
    got, ref = _adj_case(32, nt, "points", scheme=scheme)
    e2 = rel_l2(got, ref)
    print(f"Nt = {nt} {scheme}: forward {e1:.3e}, adjoint {e2:.3e}")
    assert e1 < TOL_OP and e2 < TOL_OP


def test_64_cubed_forward_adjoint():
    got, ref = _fwd_case(64, 80, "hadamard")
    e1 = rel_l2(got, ref)
    got, ref = _adj_case(64, 80, "points")
    e2 = rel_l2(got, ref)
    print(f"64^3 nt=80: forward sHd {e1:.3e}, adjoint rSP {e2:.3e}")
    assert e1 < TOL_OP and e2 < TOL_OP


@pytest.mark.parametrize("scheme", ["line", "slab"])
@pytest.mark.parametrize("kind", ["points", "hadamard", "full"])
def test_gpu_adjoint_identity(kind, scheme):
    """<C A x, y> = <x, A^T C^T y> on the GPU itself (FP32 storage, FP64 dot products)."""
    from paper_1605_00133_amd import pat as P
    n, nt = 32, 120
    smp = oracle_sampling(kind, n)
    plan = gpu_plan(n, nt, smp)
    plan.set_scheme(scheme)
    x = gaussian_volume((n, n, n), 11)
    y = gaussian_data((nt, smp.mc), 12)
    f = empty(plan.data_shape)
    p = empty(plan.vol_shape)
    P.pat_forward(plan, to_dev(x), f)
    P.pat_adjoint(plan, to_dev(y), p)
    fh, ph = to_host(f), to_host(p)
    lhs = float(np.vdot(fh, y))
    rhs = float(np.vdot(x, ph))
    # random vectors make <CAx, y> small by chance; scale by the Cauchy-Schwarz bound instead
    scale = np.linalg.norm(fh) * np.linalg.norm(y)
    rel = abs(lhs - rhs) / scale
    print(f"GPU adjoint identity {kind} {scheme}: |lhs-rhs|/(|CAx||y|) = {rel:.3e}, |lhs-rhs|/|lhs| = {abs(lhs - rhs) / abs(lhs):.3e}")
    assert rel < 1e-6


@pytest.mark.parametrize("kind", ["points", "hadamard", "full"])
def test_sampling_operators_alone(kind):
    from paper_1605_00133_amd import pat as P
    n, nt = 32, 7
    smp = oracle_sampling(kind, n)
    plan = gpu_plan(n, nt, smp)
    s = gaussian_data((nt, n, n), 21)
    f = empty(plan.data_shape)
    P.pat_sample(plan, to_dev(s), f)
    ref = apply_c(s.astype(np.float32).astype(np.float64), smp)
    got = to_host(f)
    if kind == "hadamard":
        assert rel_l2(got, ref) < 1e-6
    else:
        assert np.array_equal(got, ref)           # gathers move bits unchanged
    r = gaussian_data((nt, smp.mc), 22)
    s2 = empty(plan.plane_shape)
    P.pat_sample_adjoint(plan, to_dev(r), s2)
    ref = apply_ct(r.astype(np.float32).astype(np.float64), smp, n, n)
    got = to_host(s2)
    if kind == "hadamard":
        assert rel_l2(got, ref) < 1e-6
    else:
        assert np.array_equal(got, ref)


def test_operator_is_deterministic():
    from paper_1605_00133_amd import pat as P
    n, nt = 32, 100
    smp = oracle_sampling("hadamard", n)
    plan = gpu_plan(n, nt, smp)
    x = to_dev(phantom(n))
    a, b = empty(plan.data_shape), empty(plan.data_shape)
    P.pat_forward(plan, x, a)
    P.pat_forward(plan, x, b)
    assert np.array_equal(to_host(a), to_host(b))


@pytest.mark.parametrize("kind,scheme", [("points", "line"), ("hadamard", "line"), ("full", "slab")])
def test_sensor_sensitivity_matches_oracle(kind, scheme):
    """C W_s A and A^T W_s C^T (eq. FwdSenVar, log-normal weights sigma = 0.2) against the FP64 oracle;
    clearing the weights restores the ideal-sensor operator bit for bit."""
    import torch
    from oracle.solvers import MeasuredOperator
    from paper_1605_00133_amd import pat as P
    from synthetic import lognormal_weights
    n, nt = 32, 60
    smp = oracle_sampling(kind, n)
    w = lognormal_weights((n, n), 0.2, 9)
    op = MeasuredOperator(oracle.WaveOperator(oracle_grid(n, nt)), smp, w)
    p0 = phantom(n)
    y = gaussian_data((nt, smp.mc), 5)
    plan = gpu_plan(n, nt, smp)
    plan.set_scheme(scheme)
    f0 = empty(plan.data_shape)
    P.pat_forward(plan, to_dev(p0), f0)
    plan.set_sensitivity(w)
    f = empty(plan.data_shape)
    p = empty(plan.vol_shape)
    P.pat_forward(plan, to_dev(p0), f)
    P.pat_adjoint(plan, to_dev(y), p)
    ef, ea = rel_l2(to_host(f), op.forward(p0)), rel_l2(to_host(p), op.adjoint(y))
    print(f"W_s {kind} {scheme}: forward {ef:.2e}, adjoint {ea:.2e}")
    assert ef < 1e-5 and ea < 1e-5
    plan.set_sensitivity(None)
    f1 = empty(plan.data_shape)
    P.pat_forward(plan, to_dev(p0), f1)
    assert torch.equal(f0, f1)


@pytest.mark.parametrize("n,nt,kind", [(32, 60, "points"), (32, 40, "hadamard"), (16, 1, "full"), (16, 30, "full")])
def test_time_reversal_matches_oracle(n, nt, kind):
    """p = A^< C^T y (eq. TRnum, Dirichlet data on the detection plane) against the FP64 oracle
    (pinned by its dense 8^3 matrix), FP64 butterflies, within 1e-5; the output's plane z = 0
    is the first datum."""
    from paper_1605_00133_amd import pat as P
    smp = oracle_sampling(kind, n)
    op = oracle.WaveOperator(oracle_grid(n, nt, pml=4))
    y = gaussian_data((nt, smp.mc), 6)
    ref = op.time_reversal(apply_ct(y, smp, n, n))
    plan = gpu_plan(n, nt, smp, pml=4)
    p = empty(plan.vol_shape)
    P.pat_time_reversal(plan, to_dev(y), p)
    got = to_host(p)
    err = rel_l2(got, ref)
    print(f"time reversal {n}^3 nt={nt} {kind}: rel L2 {err:.2e}")
    assert err < 1e-5
    assert rel_l2(got[0], ref[0]) < 1e-6


@pytest.mark.parametrize("kind", ["points", "full"])
def test_heterogeneous_sound_speed_matches_oracle(kind):
    """Data generation in a 5 % perturbed medium (Sec. 5.3): C A_c p0 with p = c(x)^2 sum rho and the
    k-space reference speed max c (the grid's c0) against the FP64 oracle within 1e-5; the adjoint
    and time reversal refuse a heterogeneous plan; clearing the field restores the line scheme."""
    import torch
    from oracle.solvers import MeasuredOperator
    from paper_1605_00133_amd import pat as P
    from synthetic import sound_speed_field
    n, nt = 32, 60
    p0 = phantom(n)
    c = sound_speed_field(p0, 1500.0, 0.05, 4)
    cmax = float(c.astype(np.float32).max())
    smp = oracle_sampling(kind, n)
    ref = MeasuredOperator(oracle.WaveOperator(oracle_grid(n, nt, c0=cmax), c=c.astype(np.float32)), smp).forward(p0)
    plan = gpu_plan(n, nt, smp, c0=cmax)
    f0 = empty(plan.data_shape)
    P.pat_forward(plan, to_dev(p0), f0)
    plan.set_sound_speed(c)
    f = empty(plan.data_shape)
    P.pat_forward(plan, to_dev(p0), f)
    err = rel_l2(to_host(f), ref)
    diff = rel_l2(to_host(f), to_host(f0))
    print(f"heterogeneous medium {kind}: rel L2 vs oracle {err:.2e} (differs from homogeneous by {diff:.2e})")
    assert err < 1e-5 and diff > 1e-3
    with pytest.raises(P.PatError) as e:
        P.pat_adjoint(plan, f, empty(plan.vol_shape))
    assert e.value.status == 2
    plan.set_sound_speed(None)
    f1 = empty(plan.data_shape)
    P.pat_forward(plan, to_dev(p0), f1)
    assert torch.equal(f1, f0)
