"""Pins of the FP64 oracle's forward operator A and adjoint A^T (CPU only)."""

import json
import math
import os

import numpy as np
import pytest

from oracle import Grid, WaveOperator, nt_rule, pml_factors, wavenumbers, kappa_grid
from oracle.dense import dense_forward_matrix
from oracle.sampling import Sampling, apply_c, apply_ct
from synthetic import gaussian_blob

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small_grid(n=16, nt=24, pml=0, **kw):
    return Grid(n, n, n, dx=1e-4, c0=1500.0, dt=2e-8, nt=nt, pml_size=pml, **kw)


def test_table2_arithmetic():
    """Table 2 (Tumor1/2): CFL 0.3, 740 samples, 4.8 MHz spatial Nyquist rate."""
    t = json.load(open(os.path.join(GOLDEN, "table2_tumor_model.json")))
    cfl = t["c0_m_per_s"] * t["dt_s"] / t["dx_m"]
    assert abs(cfl - 0.3) < 1e-12
    assert nt_rule(t["n"], t["dx_m"], t["c0_m_per_s"], t["dt_s"]) == t["mt"]
    assert t["n"] * t["n"] == t["m_sensor"]
    assert abs(t["c0_m_per_s"] / (2 * t["dx_m"]) - t["nyquist_hz_printed"]) < 1.0


def test_wavenumbers_nyquist_negative():
    k = wavenumbers(8, 1.0)
    assert np.allclose(k, 2 * np.pi * np.array([0, 1, 2, 3, -4, -3, -2, -1]) / 8)


def test_kappa_is_sinc():
    g = small_grid(8)
    kap = kappa_grid(g)
    assert kap[0, 0, 0] == 1.0
    k = wavenumbers(8, g.dx)[1]
    x = g.c0 * g.dt * k / 2
    assert abs(kap[0, 0, 1] - math.sin(x) / x) < 1e-15


def test_pml_profile_hand_values():
    """exp(-alpha (c0/dx) d^4 dt/2) with d = 1 - dist/P; values worked by hand."""
    g = Grid(32, 32, 32, dx=1e-4, c0=1500.0, dt=2e-8, nt=2, pml_size=8, pml_alpha=2.0)
    f = pml_factors(g)
    s = 2.0 * 1500.0 / 1e-4 * 2e-8 / 2.0     # alpha (c0/dx) dt/2 = 0.3
    # x axis, collocated i = 0: distance 1/2 to the seam at -1/2 -> d = 1 - 1/16
    assert abs(f["b"][0][0] - math.exp(-s * (15 / 16) ** 4)) < 1e-15
    # staggered i = 31 sits on the seam (31.5 == -0.5 mod 32) -> d = 1
    assert abs(f["a"][0][31] - math.exp(-s)) < 1e-15
    # interior points are untouched
    assert f["b"][0][8] == 1.0 and f["b"][0][23] == 1.0 and f["a"][0][7] == 1.0
    # z axis: seam at N - P - 1/2 = 23.5, sensor plane z = 0 lies outside the layer
    assert f["b"][2][0] == 1.0 and f["b"][2][15] == 1.0
    assert abs(f["a"][2][23] - math.exp(-s)) < 1e-15
    assert abs(f["b"][2][16] - math.exp(-s * (1 / 16) ** 4)) < 1e-15


@pytest.mark.parametrize("n,nt", [(16, 40), (32, 30)])
def test_closed_form_without_pml(n, nt):
    """Without PML the scheme is exact: plane n of A p0 is S IFFT(cos(c0|k| n dt) FFT p0)."""
    g = small_grid(n, nt)
    rng = np.random.default_rng(11)
    p0 = rng.standard_normal(g.shape)
    s = WaveOperator(g).forward_planes(p0)
    k = [wavenumbers(n, g.dx)]
    kabs = np.sqrt(k[0][:, None, None] ** 2 + k[0][None, :, None] ** 2 + k[0][None, None, :] ** 2)
    P0 = np.fft.fftn(p0)
    ref = np.stack([np.fft.ifftn(np.cos(g.c0 * kabs * i * g.dt) * P0).real[0] for i in range(nt)])
    assert np.linalg.norm(s - ref) / np.linalg.norm(ref) < 1e-12


def test_radial_dalembert_free_space():
    """Gaussian p0 = g(r): p(r,t) = [(r-ct) g(r-ct) + (r+ct) g(r+ct)] / (2r) before any image arrives."""
    n, nt, sig = 64, 120, 2.0
    g = small_grid(n, nt)
    src = (12.0, 32.0, 32.0)
    p0 = gaussian_blob(g.shape, src, sig)
    s = WaveOperator(g).forward_planes(p0)
    yy, xx = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    near = (np.abs(yy - src[1]) <= 16) & (np.abs(xx - src[2]) <= 16)
    r = np.sqrt(src[0] ** 2 + (yy - src[1]) ** 2 + (xx - src[2]) ** 2)[near]
    gfun = lambda q: np.exp(-q * q / (2 * sig * sig))
    err = 0.0
    for i in range(nt):
        ct = g.c0 * i * g.dt / g.dx
        exact = ((r - ct) * gfun(r - ct) + (r + ct) * gfun(r + ct)) / (2 * r)
        err = max(err, np.max(np.abs(s[i][near] - exact)))
    peak = np.max(np.abs(s[:, near]))
    assert peak > 0.05
    assert err / peak < 1e-6


@pytest.mark.parametrize("pml", [0, 2])
def test_dense_bruteforce_8cubed(pml):
    """A from explicit DFT-sum matrices equals the FFT oracle; its transpose equals the adjoint."""
    g = small_grid(8, 48, pml=pml)
    A = dense_forward_matrix(g)
    op = WaveOperator(g)
    rng = np.random.default_rng(5)
    for _ in range(3):
        x = rng.standard_normal(g.shape)
        ref = A @ x.ravel()
        assert np.linalg.norm(op.forward_planes(x).ravel() - ref) / np.linalg.norm(ref) < 1e-12
        y = rng.standard_normal((g.nt, 8, 8))
        ref = A.T @ y.ravel()
        assert np.linalg.norm(op.adjoint_planes(y).ravel() - ref) / np.linalg.norm(ref) < 1e-12


def _samplings(n_pix):
    return [Sampling.full(n_pix), Sampling.points(n_pix, n_pix // 4, 2),
            Sampling.hadamard(n_pix, n_pix // 8, 4)]


@pytest.mark.parametrize("n,nt,pml", [(8, 30, 2), (32, 40, 0), (32, 40, 8)])
def test_adjoint_identity(n, nt, pml):
    g = small_grid(n, nt, pml=pml)
    op = WaveOperator(g)
    rng = np.random.default_rng(7)
    for smp in _samplings(n * n):
        x = rng.standard_normal(g.shape)
        y = rng.standard_normal((nt, smp.mc))
        lhs = np.vdot(apply_c(op.forward_planes(x), smp), y)
        rhs = np.vdot(x, op.adjoint_planes(apply_ct(y, smp, n, n)))
        assert abs(lhs - rhs) / abs(lhs) < 1e-12


def test_adjoint_identity_64_short():
    g = small_grid(64, 12, pml=8)
    op = WaveOperator(g)
    rng = np.random.default_rng(8)
    x = rng.standard_normal(g.shape)
    y = rng.standard_normal((12, 64, 64))
    lhs = np.vdot(op.forward_planes(x), y)
    rhs = np.vdot(x, op.adjoint_planes(y))
    assert abs(lhs - rhs) / abs(lhs) < 1e-12


def test_independent_of_rho0():
    rng = np.random.default_rng(9)
    x = rng.standard_normal((16, 16, 16))
    s1 = WaveOperator(small_grid(16, 20, pml=4)).forward_planes(x)
    s2 = WaveOperator(small_grid(16, 20, pml=4, rho0=1000.0)).forward_planes(x)
    assert np.linalg.norm(s1 - s2) / np.linalg.norm(s1) < 1e-12


def test_pml_suppresses_wraparound():
    """A pulse leaving through the PML must not come back: compare with a larger PML-free domain."""
    n, big, nt = 32, 64, 100
    src = (6.0, 16.0, 16.0)
    g = small_grid(n, nt, pml=8)
    s = WaveOperator(g).forward_planes(gaussian_blob(g.shape, src, 1.5))
    gb = small_grid(big, nt, pml=0)
    off = (big - n) // 2
    sb = WaveOperator(gb).forward_planes(gaussian_blob(gb.shape, (src[0], src[1] + off, src[2] + off), 1.5))
    sb = sb[:, off:off + n, off:off + n]
    core = (slice(None), slice(8, 24), slice(8, 24))
    rel = np.linalg.norm(s[core] - sb[core]) / np.linalg.norm(sb[core])
    # the big domain has no wrap-around within nt steps (its images are > 50 cells away)
    print("PML reflection (rel L2 on the sensor core):", rel)
    assert rel < 1e-2         # better than -40 dB


@pytest.mark.parametrize("kind", ["points", "hadamard"])
def test_sensor_sensitivity_weights(kind):
    """eq. FwdSenVar: C W_s A. W_s = I changes nothing; each sampled pixel's series is its
    unweighted series times that pixel's weight (random points); the weighted pair stays
    an exact transpose (adjoint identity, 1e-12)."""
    from oracle.solvers import MeasuredOperator
    from synthetic import gaussian_data, lognormal_weights
    g = Grid(16, 16, 16, dx=1e-4, c0=1500.0, dt=2e-8, nt=30, pml_size=4)
    wave = WaveOperator(g)
    smp = Sampling.points(256, 64, 2) if kind == "points" else Sampling.hadamard(256, 32, 4)
    w = lognormal_weights((16, 16), 0.2, 9)
    x = gaussian_data(g.shape, 1)
    plain, ones, wtd = MeasuredOperator(wave, smp), MeasuredOperator(wave, smp, np.ones((16, 16))), \
        MeasuredOperator(wave, smp, w)
    assert np.array_equal(ones.forward(x), plain.forward(x))
    if kind == "points":
        assert np.allclose(wtd.forward(x), plain.forward(x) * w.ravel()[smp.idx][None, :], rtol=1e-13, atol=1e-15)
    y = gaussian_data((30, smp.mc), 2)
    lhs = float(np.vdot(wtd.forward(x), y))
    rhs = float(np.vdot(x, wtd.adjoint(y)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


@pytest.mark.parametrize("pml", [0, 2])
def test_time_reversal_dense_bruteforce_8cubed(pml):
    """Time reversal (eq. TRnum) against its dense matrix built from explicit DFT sums
    (no FFT library), 1e-12; the output's sensor plane is the first datum; linear."""
    from oracle.dense import dense_time_reversal_matrix
    from synthetic import gaussian_data
    g = Grid(8, 8, 8, dx=1e-4, c0=1500.0, dt=2e-8, nt=12, pml_size=pml)
    op = WaveOperator(g)
    y = gaussian_data((12, 8, 8), 4)
    got = op.time_reversal(y)
    ref = (dense_time_reversal_matrix(g) @ y.ravel()).reshape(g.shape)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.allclose(got[0], y[0], rtol=1e-14, atol=1e-14)
    assert np.allclose(op.time_reversal(2.5 * y), 2.5 * got, rtol=1e-13, atol=1e-13)
    assert not np.allclose(got[1:], 0.0)


def test_heterogeneous_sound_speed_dense_bruteforce():
    """A with a sound-speed field (Sec. 5.3): a constant field equals the homogeneous operator;
    a 5 % perturbed field matches its dense 8^3 matrix from explicit DFT sums (1e-12) and
    changes the data by a few percent."""
    from synthetic import gaussian_data, sound_speed_field
    g = Grid(8, 8, 8, dx=1e-4, c0=1500.0, dt=2e-8, nt=14, pml_size=2)
    x = gaussian_data(g.shape, 3)
    hom = WaveOperator(g).forward_planes(x)
    assert np.array_equal(WaveOperator(g, c=np.full(g.shape, 1500.0)).forward_planes(x), hom)
    c = sound_speed_field(np.abs(x), 1500.0, 0.05, 1, smooth=1.0)
    assert abs(np.abs(c - 1500.0).max() - 75.0) < 1e-9 and abs(c.mean() - 1500.0) < 1e-9
    got = WaveOperator(g, c=c).forward_planes(x)
    ref = (dense_forward_matrix(g, c) @ x.ravel()).reshape(got.shape)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    d = np.linalg.norm(got - hom) / np.linalg.norm(hom)
    assert 1e-3 < d < 0.5
