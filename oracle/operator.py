"""Forward operator A and its exact discrete adjoint A^T (FP64, plain FFTs).

Oracle module: test infrastructure only, never called by the GPU path.

A maps the initial pressure p0 (eq. PATfwd: p(t=0) = p0, dp/dt(t=0) = 0) to
the pressure on the detection plane at the sampling times (Sec. 4.3: A maps
p0 to the first voxel layer at every time step). The scheme is the k-space
pseudospectral method the paper cites, written here with

  staggered spectral derivatives
     Dplus_xi  = IFFT[ i k_xi exp(+i k_xi dx/2) kappa FFT[.] ]   (value at xi + dx/2)
     Dminus_xi = IFFT[ i k_xi exp(-i k_xi dx/2) kappa FFT[.] ]   (value at xi - dx/2)
  split-field first-order system with PML factors a (staggered), b (collocated)
     u_xi   <- a_xi (a_xi u_xi   - dt/rho0   Dplus_xi p)
     rho_xi <- b_xi (b_xi rho_xi - dt rho0   Dminus_xi u_xi)
     p       = c0^2 (rho_x + rho_y + rho_z)
  initial condition rho_xi = p0/(3 c0^2), u_xi = (dt/(2 rho0)) Dplus_xi p0,
  which realises dp/dt(0) = 0; sample n is the plane z = 0 of p at t = n dt.

The adjoint is derived by transposing that recurrence step by step, using that
both multipliers are Hermitian so the derivative matrices are real and
(Dplus_xi)^T = -Dminus_xi. Every derivative here is a full complex 3D FFT of a
real array followed by taking the real part, so nothing depends on real-FFT
packing conventions.
"""

import numpy as np
import scipy.fft as sfft

from .grid import wavenumbers, kappa_grid, pml_factors


def _workers():
    """FFT threads: the host's cores, capped by OMP_NUM_THREADS when it is set."""
    import os
    n = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


class WaveOperator:
    """A: R^{Nz x Ny x Nx} -> R^{Nt x Ny x Nx} (detection-plane time series)."""

    def __init__(self, grid, workers=None, c=None):
        """c: optional sound-speed field [Nz][Ny][Nx] (the no-inverse-crime data model of
        Sec. 5.3); the pressure is then p = c(x)^2 sum_xi rho_xi and the initial densities
        p0 / (3 c(x)^2), while the k-space correction keeps the grid's c0 as the reference
        speed. None: homogeneous c0 everywhere."""
        self.g = grid
        self.workers = workers or _workers()
        self.c2 = None if c is None else np.asarray(c, dtype=np.float64).reshape(grid.shape) ** 2
        g = grid
        kap = kappa_grid(g)
        ks = (wavenumbers(g.nx, g.dx)[None, None, :],
              wavenumbers(g.ny, g.dx)[None, :, None],
              wavenumbers(g.nz, g.dx)[:, None, None])
        self.mplus = [1j * k * np.exp(+1j * k * g.dx / 2.0) * kap for k in ks]
        self.mminus = [1j * k * np.exp(-1j * k * g.dx / 2.0) * kap for k in ks]
        pml = pml_factors(g)
        # broadcastable PML factors per component xi = x, y, z
        self.a = [pml["a"][0][None, None, :], pml["a"][1][None, :, None], pml["a"][2][:, None, None]]
        self.b = [pml["b"][0][None, None, :], pml["b"][1][None, :, None], pml["b"][2][:, None, None]]

    # -- spectral derivatives -------------------------------------------------
    def _apply(self, mult, f):
        F = sfft.fftn(f, workers=self.workers)
        return sfft.ifftn(mult * F, workers=self.workers).real

    def dplus(self, f, xi):
        return self._apply(self.mplus[xi], f)

    def dminus(self, f, xi):
        return self._apply(self.mminus[xi], f)

    # -- A ---------------------------------------------------------------------
    def forward_planes(self, p0, nsteps=None):
        """Pressure on the plane z = 0 at t = n dt, n = 0..Nt-1 -> [Nt][Ny][Nx]."""
        g = self.g
        nt = g.nt if nsteps is None else nsteps
        p0 = np.asarray(p0, dtype=np.float64)
        c2 = g.c0 * g.c0 if self.c2 is None else self.c2
        rho = [p0 / (3.0 * c2) for _ in range(3)]
        u = [(g.dt / (2.0 * g.rho0)) * self.dplus(p0, xi) for xi in range(3)]
        s = np.empty((nt, g.ny, g.nx))
        p = p0.copy()
        s[0] = p[0]
        for n in range(nt - 1):
            for xi in range(3):
                u[xi] = self.a[xi] * (self.a[xi] * u[xi] - (g.dt / g.rho0) * self.dplus(p, xi))
            for xi in range(3):
                rho[xi] = self.b[xi] * (self.b[xi] * rho[xi] - g.dt * g.rho0 * self.dminus(u[xi], xi))
            p = c2 * (rho[0] + rho[1] + rho[2])
            s[n + 1] = p[0]
        return s

    # -- A^T -------------------------------------------------------------------
    def adjoint_planes(self, y):
        """Exact transpose of forward_planes: [Nt][Ny][Nx] -> [Nz][Ny][Nx] (homogeneous c0)."""
        if self.c2 is not None:
            raise NotImplementedError("the adjoint is built for the homogeneous sound speed only")
        g = self.g
        y = np.asarray(y, dtype=np.float64)
        nt = y.shape[0]
        c2 = g.c0 * g.c0

        def src(n):                       # c0^2 S^T y^n as a volume
            v = np.zeros(g.shape)
            v[0] = c2 * y[n]
            return v

        rhoh = [src(nt - 1) for _ in range(3)]   # adjoint of rho_xi after the last step
        v = [np.zeros(g.shape) for _ in range(3)]  # adjoint of u_xi after the last step
        for n in range(nt - 2, -1, -1):
            # transpose of  rho_xi' = b^2 rho_xi - b dt rho0 Dminus_xi u_xi'
            uh = [v[xi] + g.dt * g.rho0 * self.dplus(self.b[xi] * rhoh[xi], xi) for xi in range(3)]
            # transpose of  u_xi' = a^2 u_xi - a (dt/rho0) Dplus_xi (c0^2 sum rho)
            q = sum(self.dminus(self.a[xi] * uh[xi], xi) for xi in range(3))
            q = c2 * (g.dt / g.rho0) * q
            s = src(n)
            rhoh = [self.b[xi] * self.b[xi] * rhoh[xi] + q + s for xi in range(3)]
            v = [self.a[xi] * self.a[xi] * uh[xi] for xi in range(3)]
        # transpose of the initial condition
        p = (rhoh[0] + rhoh[1] + rhoh[2]) / (3.0 * c2)
        p -= (g.dt / (2.0 * g.rho0)) * sum(self.dminus(v[xi], xi) for xi in range(3))
        return p

    # -- time reversal A^< (eq. TRnum) ----------------------------------------------------------
    def time_reversal(self, y):
        """A^< applied to a plane series y [Nt][Ny][Nx]: the same recurrence run from zero
        fields with the time-reversed series imposed on the detection plane as a Dirichlet
        condition (Sec. 4.4): after the density update of every step (and at the start) each
        density component on z = 0 is set to y^(Nt-1-n) / (3 c0^2), so that the pressure there
        equals the datum; the output is the pressure field after the last step (whose plane
        z = 0 is y^0)."""
        g = self.g
        if self.c2 is not None:
            raise NotImplementedError("time reversal is built for the homogeneous sound speed only")
        y = np.asarray(y, dtype=np.float64)
        nt = y.shape[0]
        c2 = g.c0 * g.c0
        rho = [np.zeros(g.shape) for _ in range(3)]
        for xi in range(3):
            rho[xi][0] = y[nt - 1] / (3.0 * c2)
        u = [np.zeros(g.shape) for _ in range(3)]
        p = c2 * (rho[0] + rho[1] + rho[2])
        for n in range(nt - 1):
            for xi in range(3):
                u[xi] = self.a[xi] * (self.a[xi] * u[xi] - (g.dt / g.rho0) * self.dplus(p, xi))
            for xi in range(3):
                rho[xi] = self.b[xi] * (self.b[xi] * rho[xi] - g.dt * g.rho0 * self.dminus(u[xi], xi))
                rho[xi][0] = y[nt - 2 - n] / (3.0 * c2)
            p = c2 * (rho[0] + rho[1] + rho[2])
        return p
