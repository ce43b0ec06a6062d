"""The paper-scale reconstruction workload on the GPU, its regularisation
parameter, and the time-to-target measurement of plain TV+Br.

Workload (the Tumor1/2 grid of Table 2 with synthetic vessels in place of the
unavailable phantoms): 128^3 grid incl. an 8-cell PML, dx = 100 um,
c0 = 1500 m/s, dt = 20 ns (CFL 0.3), Nt = 740, the 128 x 128 detection plane;
p0 = 24 random vessels of radius 1-4 voxels (seed 1); random 12.5 % single
points (2048 of 16384 pixels, seed 2) or 2048 rows of a scrambled Hadamard
matrix (seeds 4/5); f = C A p0 + sigma N(0, 1), sigma = 0.01 max |C A p0|
(noise seed 3); L by 10 power steps from N(0, 1) (seed 8).

lambda_TV+ is chosen once by the discrepancy principle (eq. DiscPr, Sec. 5.2:
kappa = 1.25 within 0.01) and frozen in synthetic.CONFIGS["paper"]; TV+Br uses
lambda_Br = 10 lambda_TV+ (Sec. 5.2) for 5 Bregman steps of 50 FISTA
iterations. The principle is applied to TV+ solved closer to convergence, by
200 FISTA iterations of 50 PDHG steps: after 50 iterations even lambda -> 0
leaves the discrepancy at 1.6 (rSP) / 2.2 (sHd) of the noise level, so the
equation has no root at that budget; after 200 it falls to about 1.1.

Time to target: the plain TV+Br run logs PSNR (eq. PSNR) and wall time after
every FISTA iteration; its target is its final PSNR minus 0.5 dB, and its time
to target the first logged time at which its PSNR reaches that value.

Every computation runs in libpat (pat_forward, pat_power_iteration,
pat_reconstruct); this module sets up inputs and reads logs.

CLI: python -m paper_1605_00133_amd.workload --calibrate [--sampling points|hadamard]
     prints the discrepancy-principle lambda_TV+ as JSON.
"""

import json
import math
import sys

import numpy as np
import torch

from . import pat as P
from .dp import bregman_stop, tv_lambda


def paper_problem(sampling="points", n=128, nt=740, device="cuda:0", n_power=10):
    """Plan, phantom, data and step-size estimate of the paper-scale workload (dict)."""
    from synthetic import CONFIGS, gaussian_data, gaussian_volume, vessel_phantom
    cfg = CONFIGS["paper"]
    dev = torch.device(device)
    npix = n * n
    mc = npix // 8
    if sampling == "points":
        idx, perm = P.pat_make_rsp_mask(npix, mc, cfg["mask_seed"]), None
    elif sampling == "hadamard":
        perm, idx = P.pat_make_shd_pattern(npix, mc, cfg["hadamard_seed"])
    else:
        raise ValueError(f"unknown sampling {sampling!r}")
    grid = P.make_grid(n, n, n, cfg["dx"], cfg["c0"], cfg["dt"], nt, cfg["pml"], cfg["pml_alpha"])
    plan = P.Plan(grid, sampling, mc, idx, perm, device=device)
    p0_h = vessel_phantom((n, n, n), cfg["pml"], cfg["n_vessels"], cfg["r_min"], cfg["r_max"], cfg["phantom_seed"])
    p0 = torch.from_numpy(p0_h.astype(np.float32)).to(dev)
    f = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
    P.pat_forward(plan, p0, f)
    torch.cuda.synchronize(dev)
    sigma = cfg["noise_rel"] * float(f.abs().max())
    f += sigma * torch.from_numpy(gaussian_data(plan.data_shape, cfg["noise_seed"]).astype(np.float32)).to(dev)
    x0 = torch.from_numpy(gaussian_volume(plan.vol_shape, 8).astype(np.float32)).to(dev)
    L = P.pat_power_iteration(plan, x0, n_power)
    lam_tv = (cfg.get("lam_tv") or {}).get(sampling) if (n, nt) == (cfg["n"], cfg["nt"]) else None
    return {"plan": plan, "p0": p0, "p0_host": p0_h, "f": f, "sigma": sigma, "L": L, "n": n, "nt": nt,
            "sampling": sampling, "mc": mc, "idx": idx, "perm": perm, "lam_tv": lam_tv,
            "lam_br": None if lam_tv is None else cfg["br_factor"] * lam_tv}


def calibrate(prob, n_inner=200, n_prox=50, kappa=1.25, tol=0.01, lo=1e-5, hi=1e-3):
    """lambda_TV+ by the discrepancy principle on this problem, searched from the interval
    [lo, hi] * sigma sqrt(Nt M_c); returns (lam, discrepancy, history)."""
    plan, f, sigma, L = prob["plan"], prob["f"], prob["sigma"], prob["L"]
    s = sigma * math.sqrt(plan.data_shape[0] * plan.data_shape[1])
    p = torch.empty(plan.vol_shape, dtype=torch.float32, device=f.device)
    return tv_lambda(plan, f, p, sigma, L, lo * s, hi * s, n_inner=n_inner, n_prox=n_prox, kappa=kappa, tol=tol)


def target_time(psnr, t_ms, margin_db=0.5, final=None):
    """(target PSNR, first logged time [ms] at which psnr >= target, its iteration index)."""
    final = float(psnr[-1]) if final is None else float(final)
    target = final - margin_db
    for i, (q, t) in enumerate(zip(psnr, t_ms)):
        if q >= target:
            return target, float(t), i
    return target, None, None


def tv_bregman_curve(prob, n_outer=5, n_inner=50, n_prox=50, margin_db=0.5):
    """The plain TV+Br run with PSNR and wall time logged per FISTA iteration."""
    plan, f, p0 = prob["plan"], prob["f"], prob["p0"]
    p = torch.empty(plan.vol_shape, dtype=torch.float32, device=f.device)
    torch.cuda.synchronize(f.device)
    out = P.pat_reconstruct(plan, f, p, prob["lam_br"], prob["L"], n_outer=n_outer, n_inner=n_inner,
                            n_prox=n_prox, bc="dirichlet", restart=True, p_ref=p0)
    psnr, t_ms = out["psnr"], out["t_ms"]
    target, t_target, i_target = target_time(psnr, t_ms, margin_db)
    n_data = plan.data_shape[0] * plan.data_shape[1]
    flags = out["flags"]
    return {"p": p, "psnr": psnr, "t_ms": t_ms, "final_psnr_db": float(psnr[-1]), "best_psnr_db": float(psnr.max()),
            "total_ms": float(t_ms[-1]), "target_psnr_db": target, "t_target_ms": t_target,
            "target_iteration": None if i_target is None else int(i_target) + 1,
            "iterations": int(len(psnr)), "restarts": int((flags > 0).sum()),
            "pairs": 0.5 * (2 * len(flags) + int(flags.sum()) + int((flags > 0).sum())),
            "psnr_per_outer": [float(psnr[(k + 1) * n_inner - 1]) for k in range(n_outer)],
            "t_ms_per_outer": [float(t_ms[(k + 1) * n_inner - 1]) for k in range(n_outer)],
            "bregman_discrepancy": [float(r / (math.sqrt(n_data) * prob["sigma"])) for r in out["bregman_residual"]],
            "bregman_dp_stop": bregman_stop(out["bregman_residual"], n_data, prob["sigma"])}


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="Paper-scale workload: discrepancy-principle lambda, TV+Br curve.")
    ap.add_argument("--sampling", choices=["points", "hadamard"], default="points")
    ap.add_argument("--calibrate", action="store_true", help="run the discrepancy-principle search for lambda_TV+")
    ap.add_argument("--curve", action="store_true", help="run TV+Br (5 x 50) with the frozen lambda and log PSNR")
    a = ap.parse_args(argv)
    prob = paper_problem(a.sampling)
    res = {"sampling": a.sampling, "L": prob["L"], "sigma": prob["sigma"]}
    if a.calibrate:
        lam, d, hist = calibrate(prob)
        res.update({"lam_tv": lam, "discrepancy": d, "evaluations": len(hist),
                    "history": [[float(x), float(y)] for x, y in hist]})
        print(f"lambda_TV+ = {lam:.6e}, discrepancy {d:.4f} after {len(hist)} reconstructions", file=sys.stderr)
    if a.curve:
        c = tv_bregman_curve(prob)
        res.update({k: v for k, v in c.items() if k not in ("p", "psnr", "t_ms")})
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
