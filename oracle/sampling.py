"""Sub-sampling operators C and C^T, and the seeded index generators.

Oracle module: test infrastructure only, never called by the GPU path.

The paper models each measurement as the detection-plane pressure weighted by
a window function and integrated over the plane (eq. GenScan), sampled at
every time step. Three discrete instances are used (Sec. 3.1 and 4.3):

* conventional scan: every plane voxel is a sensor (C = identity);
* random single points (rSP): M_c plane voxels chosen at random; C extracts
  their time series;
* scrambled Hadamard patterns (sHd): M_c rows of a column-scrambled +-1
  Hadamard matrix applied to the plane at every time point, implemented by a
  fast FFT-like transform.

For both sub-sampling operators the pseudo-inverse equals the transpose
(Sec. 4.4), i.e. C C^T = I, which fixes the sHd scale to 1/sqrt(n_pix).

Readings (the paper gives no generator): indices come from SplitMix64
(Steele, Lea and Flood, OOPSLA 2014) driving a Durstenfeld Fisher-Yates
shuffle with unbiased bounded draws by rejection:

    bounded(m): repeat x = next(); r = x mod m; until x - r <= 2^64 - m; return r
    shuffle(n, seed): a = [0..n); for i = n-1 down to 1: j = bounded(i+1); swap a[i], a[j]

rSP keeps the first M_c entries of shuffle(n_pix, seed), sorted ascending.
sHd uses shuffle(n_pix, seed) as the column permutation pi and the first M_c
entries of shuffle(n_pix, seed + 1), sorted, as the selected Hadamard rows.
The Hadamard matrix is Sylvester's in natural order, W[r][q] = (-1)^popcount(r & q).
"""

from dataclasses import dataclass
from typing import Optional

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15


def splitmix64_stream(seed):
    """Generator of SplitMix64 outputs for a 64-bit seed (pure Python ints)."""
    state = seed & MASK64
    while True:
        state = (state + GOLDEN_GAMMA) & MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        yield z ^ (z >> 31)


def bounded_draw(rng, m):
    """Unbiased integer in [0, m) from a 64-bit stream, by rejection."""
    limit = (1 << 64) - m
    while True:
        x = next(rng)
        r = x % m
        if x - r <= limit:
            return r


def fisher_yates(n, seed):
    """Durstenfeld shuffle of range(n) driven by SplitMix64(seed)."""
    rng = splitmix64_stream(seed)
    a = list(range(n))
    for i in range(n - 1, 0, -1):
        j = bounded_draw(rng, i + 1)
        a[i], a[j] = a[j], a[i]
    return a


def rsp_mask(n_pix, mc, seed):
    """Sorted indices of M_c distinct random plane pixels (rSP)."""
    if not (0 < mc <= n_pix):
        raise ValueError("need 0 < mc <= n_pix")
    return np.array(sorted(fisher_yates(n_pix, seed)[:mc]), dtype=np.int32)


def shd_pattern(n_pix, mc, seed):
    """(perm, rows) of a scrambled Hadamard pattern set (sHd)."""
    if n_pix <= 0 or (n_pix & (n_pix - 1)) != 0:
        raise ValueError("Hadamard patterns need a power-of-two pixel count")
    if not (0 < mc <= n_pix):
        raise ValueError("need 0 < mc <= n_pix")
    perm = np.array(fisher_yates(n_pix, seed), dtype=np.int32)
    rows = np.array(sorted(fisher_yates(n_pix, seed + 1)[:mc]), dtype=np.int32)
    return perm, rows


def fwht(x):
    """Unnormalised Walsh-Hadamard transform along the last axis (Sylvester order)."""
    y = np.array(x, dtype=np.float64, copy=True)
    n = y.shape[-1]
    h = 1
    while h < n:
        y = y.reshape(y.shape[:-1] + (n // (2 * h), 2, h))
        lo = y[..., 0, :].copy()
        hi = y[..., 1, :].copy()
        y[..., 0, :] = lo + hi
        y[..., 1, :] = lo - hi
        y = y.reshape(y.shape[:-3] + (n,))
        h *= 2
    return y


@dataclass
class Sampling:
    kind: str                      # "full", "points" or "hadamard"
    mc: int
    idx: Optional[np.ndarray] = None    # points: pixel ids; hadamard: row ids
    perm: Optional[np.ndarray] = None   # hadamard: column permutation

    @staticmethod
    def full(n_pix):
        return Sampling("full", n_pix)

    @staticmethod
    def points(n_pix, mc, seed):
        return Sampling("points", mc, idx=rsp_mask(n_pix, mc, seed))

    @staticmethod
    def hadamard(n_pix, mc, seed):
        perm, rows = shd_pattern(n_pix, mc, seed)
        return Sampling("hadamard", mc, idx=rows, perm=perm)


def apply_c(s, smp):
    """C: plane series [Nt][Ny][Nx] -> data [Nt][M_c]."""
    nt = s.shape[0]
    flat = np.asarray(s, dtype=np.float64).reshape(nt, -1)
    if smp.kind == "full":
        return flat.copy()
    if smp.kind == "points":
        return flat[:, smp.idx]
    n = flat.shape[1]
    return fwht(flat[:, smp.perm])[:, smp.idx] / np.sqrt(n)


def apply_ct(f, smp, ny, nx):
    """C^T: data [Nt][M_c] -> plane series [Nt][Ny][Nx]."""
    f = np.asarray(f, dtype=np.float64)
    nt = f.shape[0]
    n = ny * nx
    if smp.kind == "full":
        return f.reshape(nt, ny, nx).copy()
    out = np.zeros((nt, n))
    if smp.kind == "points":
        out[:, smp.idx] = f
        return out.reshape(nt, ny, nx)
    z = np.zeros((nt, n))
    z[:, smp.idx] = f
    w = fwht(z) / np.sqrt(n)        # W is symmetric
    out[:, smp.perm] = w            # transpose of the column gather
    return out.reshape(nt, ny, nx)
