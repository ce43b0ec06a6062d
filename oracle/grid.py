"""Grid, wavenumbers, k-space correction and PML profiles (FP64).

Oracle module: test infrastructure only, never called by the GPU path.

The paper discretises the domain into N = Nx*Ny*Nz voxels and propagates the
acoustic initial-value problem (eq. PATfwd) with the k-space pseudospectral
time-domain method, using a time step equal to the temporal sampling interval
(Sec. 4.3, "Discrete Forward Model"). The paper defers the details of that
scheme to its citations; the readings used here are:

* arrays are indexed [iz][iy][ix] (x fastest) and voxel (ix,iy,iz) sits at
  (ix,iy,iz)*dx; the detection plane is the first voxel layer, z = 0;
* k(m) = 2*pi*m'/(n*dx) with m' = m for m < n/2 and m - n otherwise, so the
  Nyquist bin of an even length carries the negative wavenumber;
* k-space correction kappa = sinc(c0*dt*|k|/2), sinc(0) = 1;
* a perfectly matched layer of P cells sits inside the FFT grid: on x and y a
  2P-cell slab centred on the periodic seam at -1/2, on z a 2P-cell slab
  z in [N-2P, N) so the sensor plane z = 0 lies directly in front of it;
  profile d = max(0, 1 - dist/P), sigma = alpha*(c0/dx)*d^4 and the per
  half-step factor exp(-sigma*dt/2), sampled at collocated points i (b) and at
  staggered points i+1/2 (a).
"""

from dataclasses import dataclass
import math

import numpy as np


@dataclass(frozen=True)
class Grid:
    """Discretisation parameters (Table 2 lists the paper's values)."""
    nx: int
    ny: int
    nz: int
    dx: float          # isotropic voxel size [m]
    c0: float          # homogeneous sound speed [m/s]
    dt: float          # time step = temporal sampling interval [s]
    nt: int            # number of time samples t = 0, dt, ..., (nt-1) dt
    rho0: float = 1.0  # ambient density; A does not depend on it
    pml_size: int = 8
    pml_alpha: float = 2.0

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def n_pix(self):
        return self.nx * self.ny

    @property
    def cfl(self):
        return self.c0 * self.dt / self.dx


def nt_rule(n, dx, c0, dt):
    """Number of samples needed for a wave to cross the cube diagonal once.

    With the Tumor1/2 model of Table 2 (N = 128, dx = 156.25 um, c0 = 1500 m/s,
    dt = 31.25 ns) this gives the 740 samples listed there.
    """
    return int(math.floor(math.sqrt(3.0) * n * dx / (c0 * dt))) + 1


def wavenumbers(n, dx):
    """Angular wavenumbers of an n-point periodic grid, FFT ordering."""
    m = np.arange(n, dtype=np.float64)
    m = np.where(m < n / 2, m, m - n)
    return 2.0 * np.pi * m / (n * dx)


def kappa_grid(g):
    """k-space correction sinc(c0*dt*|k|/2) on the full [kz][ky][kx] grid."""
    kx = wavenumbers(g.nx, g.dx)[None, None, :]
    ky = wavenumbers(g.ny, g.dx)[None, :, None]
    kz = wavenumbers(g.nz, g.dx)[:, None, None]
    kabs = np.sqrt(kx * kx + ky * ky + kz * kz)
    # numpy's sinc is sin(pi x)/(pi x) with sinc(0) = 1
    return np.sinc(g.c0 * g.dt * kabs / (2.0 * np.pi))


def _pml_factor(pos, n, seam, g):
    """exp(-sigma*dt/2) at (possibly fractional) positions `pos` on a periodic axis."""
    if g.pml_size == 0:
        return np.ones_like(pos)
    dist = np.abs(pos - seam) % n
    dist = np.minimum(dist, n - dist)
    d = np.maximum(0.0, 1.0 - dist / g.pml_size)
    sigma = g.pml_alpha * (g.c0 / g.dx) * d ** 4
    return np.exp(-sigma * g.dt / 2.0)


def pml_factors(g):
    """Per-axis PML factors.

    Returns dict with keys 'a' and 'b', each a tuple (fx, fy, fz) of 1D arrays;
    'b' is sampled at collocated points i and 'a' at staggered points i + 1/2.
    """
    out = {"a": [], "b": []}
    for n, axis in ((g.nx, "x"), (g.ny, "y"), (g.nz, "z")):
        seam = -0.5 if axis in ("x", "y") else n - g.pml_size - 0.5
        i = np.arange(n, dtype=np.float64)
        out["b"].append(_pml_factor(i, n, seam, g))
        out["a"].append(_pml_factor(i + 0.5, n, seam, g))
    return {k: tuple(v) for k, v in out.items()}


def interior_box(g):
    """(z0, z1, y0, y1, x0, x1): the non-PML region, half-open bounds."""
    P = g.pml_size
    return (0, g.nz - 2 * P, P, g.ny - P, P, g.nx - P)
