"""Workload parameters (plain numbers, no method arithmetic).

small   : 32^3 grid incl. 8-cell PML, dx = 100 um, c0 = 1500 m/s, dt = 20 ns
          (CFL 0.3), Nt = 190, 32x32 sensor plane at z = 0; 6 vessels of
          radius 1-2 voxels; random 25 % single-point sub-sampling (256 of
          1024 pixels); 1 % Gaussian noise; 10 FISTA iterations of TV+
          with lambda = 1e-3.
paper   : 128^3 grid, same spacing/speed/CFL, Nt = 740, 128x128 sensor plane
          (the Tumor1/2 grid and sample count of Table 2); 24 vessels of
          radius 1-4 voxels; random 12.5 % single points (2048 of 16384) or
          2048 scrambled +-1 Hadamard patterns; 1 % noise; TV + Bregman,
          5 outer x 50 inner FISTA iterations. lam_tv: the TV+ weight per
          sampling mode, chosen once by the discrepancy principle (kappa = 1.25
          within 0.01; `python -m paper_1605_00133_amd.workload --calibrate`)
          and frozen here; TV+Br uses br_factor * lam_tv. lam_tv_rel = lam_tv /
          (sigma sqrt(Nt M_c)) of the same calibration, for other phantoms of
          the workload (their own noise level sigma).
"""

CONFIGS = {
    "small": dict(n=32, dx=100e-6, c0=1500.0, dt=20e-9, nt=190, pml=8, pml_alpha=2.0,
                  n_vessels=6, r_min=1.0, r_max=2.0, phantom_seed=1,
                  sampling="points", mc=256, mask_seed=2, noise_seed=3, noise_rel=0.01,
                  lam=1e-3, n_outer=1, n_inner=10, n_prox=50),
    "paper": dict(n=128, dx=100e-6, c0=1500.0, dt=20e-9, nt=740, pml=8, pml_alpha=2.0,
                  n_vessels=24, r_min=1.0, r_max=4.0, phantom_seed=1,
                  sampling="points", mc=2048, mask_seed=2, hadamard_seed=4,
                  noise_seed=3, noise_rel=0.01,
                  lam=None, lam_tv={"points": 2.7730e-3, "hadamard": 1.6518e-3},
                  lam_tv_rel={"points": 6.3342e-4, "hadamard": 5.5343e-4}, br_factor=10.0,
                  n_outer=5, n_inner=50, n_prox=50),
}


def make_grid_params(name):
    c = CONFIGS[name]
    return dict(nx=c["n"], ny=c["n"], nz=c["n"], dx=c["dx"], c0=c["c0"], dt=c["dt"],
                nt=c["nt"], pml_size=c["pml"], pml_alpha=c["pml_alpha"])
