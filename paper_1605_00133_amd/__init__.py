"""MI355X-native hot path of compressed-sensing photoacoustic tomography.

The computation lives in libpat.so (hand-written HIP for gfx950 behind the C
ABI of include/pat.h); `pat` is its ctypes binding.
"""

from . import pat  # noqa: F401
from .pat import (Plan, PatError, lib, make_grid, pat_adjoint, pat_forward, pat_make_rsp_mask,  # noqa: F401
                  pat_make_shd_pattern, pat_plan_workspace_bytes, pat_power_iteration, pat_psnr,
                  pat_reconstruct, pat_sample, pat_sample_adjoint, pat_tv_dual_floats, pat_tv_norm,
                  pat_tv_prox)
