"""Plain FP64 CPU oracle for the compressed-sensing photoacoustic tomography
hot path (Arridge et al., "Accelerated high-resolution photoacoustic
tomography via compressed sensing").

This package is TEST INFRASTRUCTURE. Only the test-suite, the smoke check and
the CPU-baseline leg of the benchmark may import it. The GPU product path
never calls into it, and it shares no code, tables or constants with the HIP
implementation: both sides start from the paper's definitions.

Modules
  grid      grid, wavenumbers, k-space correction, PML profiles (Sec. 4.3)
  operator  forward operator A and its exact adjoint (eq. PATfwd, Sec. 4.3)
  sampling  SplitMix64 masks, scrambled Hadamard patterns, C and C^T (Sec. 3.1, 4.3)
  tv        discrete isotropic TV and its PDHG proximal operator (App. A, App. B)
  solvers   FISTA with restart/backtracking, Bregman, power iteration (App. B, Sec. 4.6)
  metrics   thresholded PSNR (eq. PSNR)
  dense     explicit-matrix brute force of A for tiny grids (pins the FFT operator)

Parity status: every function here is pinned by a `-m "not gpu"` test against a
closed form, a brute force, a library routine or an invariant; the paper's own
reconstruction PSNRs refer to phantoms that are not available, so agreement
with those printed values is "parity unpinned".
"""

from .grid import Grid, wavenumbers, kappa_grid, pml_factors, nt_rule
from .operator import WaveOperator
from .sampling import (Sampling, splitmix64_stream, bounded_draw, fisher_yates,
                       rsp_mask, shd_pattern, fwht, apply_c, apply_ct)
from .tv import grad, div, tv_value, prox_tv_pos
from .solvers import MeasuredOperator, fista, bregman, power_iteration
from .metrics import psnr, eval_region

__all__ = [
    "Grid", "wavenumbers", "kappa_grid", "pml_factors", "nt_rule",
    "WaveOperator", "Sampling", "splitmix64_stream", "bounded_draw",
    "fisher_yates", "rsp_mask", "shd_pattern", "fwht", "apply_c", "apply_ct",
    "grad", "div", "tv_value", "prox_tv_pos", "MeasuredOperator", "fista",
    "bregman", "power_iteration", "psnr", "eval_region",
]
