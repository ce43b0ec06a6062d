"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module only draws inputs (phantoms, random vectors, noise, start
vectors). It contains none of the reconstruction method's arithmetic: no
wave propagation, no sampling operator, no TV, no solver.

The paper's phantoms (micro-CT mouse-brain segmentations, Sec. 5.1) and its
experimental data are not available; random tubular vessel phantoms of the
same grid sizes stand in for them.
"""

from .phantoms import (vessel_phantom, moving_vessel_frames, gaussian_volume, gaussian_data, gaussian_blob,
                       lognormal_weights, sound_speed_field)
from .configs import CONFIGS, make_grid_params

__all__ = ["vessel_phantom", "moving_vessel_frames", "gaussian_volume", "gaussian_data", "gaussian_blob", "lognormal_weights",
           "sound_speed_field",
           "CONFIGS", "make_grid_params"]
