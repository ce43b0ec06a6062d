"""Explicit-matrix brute force of C A for tiny grids (FP64).

Oracle module: test infrastructure only, never called by the GPU path.

Builds every spectral derivative as a dense matrix from the direct DFT sum
  D[i, j] = Re( (1/N) sum_k M(k) exp(i k . (x_i - x_j)) )
(no FFT library), runs the same first-order recurrence on matrices instead of
vectors and stacks the plane rows, giving A as an (Nt*Ny*Nx) x N matrix.
It pins the FFT-based operator (derivatives, staggering, PML application,
initial condition) and, through its plain transpose, the adjoint routine.
"""

import numpy as np
import scipy.linalg

from .grid import wavenumbers, kappa_grid, pml_factors


def _dft_matrix(n):
    j = np.arange(n)
    return np.exp(-2j * np.pi * np.outer(j, j) / n)


def dense_derivatives(g):
    Fx, Fy, Fz = _dft_matrix(g.nx), _dft_matrix(g.ny), _dft_matrix(g.nz)
    F = np.kron(Fz, np.kron(Fy, Fx))            # flattening order [z][y][x]
    N = g.nx * g.ny * g.nz
    kap = kappa_grid(g)
    ks = (wavenumbers(g.nx, g.dx)[None, None, :],
          wavenumbers(g.ny, g.dx)[None, :, None],
          wavenumbers(g.nz, g.dx)[:, None, None])
    dp, dm = [], []
    for k in ks:
        for sign, out in ((+1, dp), (-1, dm)):
            m = (1j * k * np.exp(sign * 1j * k * g.dx / 2.0) * kap).ravel()
            out.append(np.real(F.conj().T @ (m[:, None] * F)) / N)
    return dp, dm


def dense_forward_matrix(g, c=None):
    """A as a dense matrix: rows (n, iy, ix), columns flattened p0; c: optional sound-speed
    field (pressure c(x)^2 sum rho, initial densities p0 / (3 c(x)^2), k-space correction
    with the grid's c0)."""
    N = g.nx * g.ny * g.nz
    npix = g.nx * g.ny
    dp, dm = dense_derivatives(g)
    pml = pml_factors(g)
    ones = (np.ones(g.nx), np.ones(g.ny), np.ones(g.nz))

    def expand(vec, axis):
        f = [ones[0][None, None, :], ones[1][None, :, None], ones[2][:, None, None]]
        shp = [(1, 1, g.nx), (1, g.ny, 1), (g.nz, 1, 1)][axis]
        f[axis] = vec.reshape(shp)
        return (f[0] * f[1] * f[2]).ravel()

    a = [expand(pml["a"][i], i) for i in range(3)]
    b = [expand(pml["b"][i], i) for i in range(3)]
    c2 = np.full(N, g.c0 ** 2) if c is None else np.asarray(c, dtype=np.float64).ravel() ** 2
    I = np.eye(N)
    R = [I / (3.0 * c2[:, None]) for _ in range(3)]
    U = [(g.dt / (2.0 * g.rho0)) * dp[i] for i in range(3)]
    P = I
    rows = [P[:npix]]
    for _ in range(g.nt - 1):
        U = [a[i][:, None] * (a[i][:, None] * U[i] - (g.dt / g.rho0) * (dp[i] @ P)) for i in range(3)]
        R = [b[i][:, None] * (b[i][:, None] * R[i] - g.dt * g.rho0 * (dm[i] @ U[i])) for i in range(3)]
        P = c2[:, None] * (R[0] + R[1] + R[2])
        rows.append(P[:npix])
    return np.vstack(rows)


def dense_time_reversal_matrix(g):
    """Time reversal A^< as a dense N x (Nt*Ny*Nx) matrix (columns: the plane series y
    flattened (n, iy, ix)), from the same explicit derivative matrices: zero fields, the
    density components on the plane z = 0 replaced by y^(Nt-1-n) / (3 c0^2) at the start
    and after every density update, the pressure field after the last step."""
    N = g.nx * g.ny * g.nz
    npix = g.nx * g.ny
    M = g.nt * npix
    dp, dm = dense_derivatives(g)
    pml = pml_factors(g)
    ones = (np.ones(g.nx), np.ones(g.ny), np.ones(g.nz))

    def expand(vec, axis):
        f = [ones[0][None, None, :], ones[1][None, :, None], ones[2][:, None, None]]
        shp = [(1, 1, g.nx), (1, g.ny, 1), (g.nz, 1, 1)][axis]
        f[axis] = vec.reshape(shp)
        return (f[0] * f[1] * f[2]).ravel()

    def inject(k):
        E = np.zeros((npix, M))
        E[np.arange(npix), k * npix + np.arange(npix)] = 1.0
        return E

    a = [expand(pml["a"][i], i) for i in range(3)]
    b = [expand(pml["b"][i], i) for i in range(3)]
    c2 = g.c0 ** 2
    R = [np.zeros((N, M)) for _ in range(3)]
    for i in range(3):
        R[i][:npix] = inject(g.nt - 1) / (3.0 * c2)
    U = [np.zeros((N, M)) for _ in range(3)]
    P = c2 * (R[0] + R[1] + R[2])
    for n in range(g.nt - 1):
        U = [a[i][:, None] * (a[i][:, None] * U[i] - (g.dt / g.rho0) * (dp[i] @ P)) for i in range(3)]
        R = [b[i][:, None] * (b[i][:, None] * R[i] - g.dt * g.rho0 * (dm[i] @ U[i])) for i in range(3)]
        for i in range(3):
            R[i][:npix] = inject(g.nt - 2 - n) / (3.0 * c2)
        P = c2 * (R[0] + R[1] + R[2])
    return P


def dense_sampling_matrix(smp, n_pix):
    if smp.kind == "full":
        return np.eye(n_pix)
    if smp.kind == "points":
        return np.eye(n_pix)[smp.idx]
    W = scipy.linalg.hadamard(n_pix).astype(np.float64)
    Pm = np.zeros((n_pix, n_pix))
    Pm[np.arange(n_pix), smp.perm] = 1.0
    return (W[smp.idx] @ Pm) / np.sqrt(n_pix)


def dense_measured_matrix(g, smp):
    """C A as a dense (Nt*M_c) x N matrix, rows ordered (n, j)."""
    A = dense_forward_matrix(g)
    Cm = dense_sampling_matrix(smp, g.nx * g.ny)
    npix = g.nx * g.ny
    blocks = [Cm @ A[n * npix:(n + 1) * npix] for n in range(g.nt)]
    return np.vstack(blocks)


class DenseOperator:
    """Same interface as solvers.MeasuredOperator, backed by a dense matrix."""

    def __init__(self, g, smp):
        self.M = dense_measured_matrix(g, smp)
        self.in_shape = g.shape
        self.out_shape = (g.nt, smp.mc)

    def forward(self, x):
        return (self.M @ np.asarray(x).ravel()).reshape(self.out_shape)

    def adjoint(self, r):
        return (self.M.T @ np.asarray(r).ravel()).reshape(self.in_shape)
