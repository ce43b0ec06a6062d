"""Benchmark: fwd+adj operator pairs/s at 128^3 inside the TV(+Bregman) FISTA loop.

A step is one FISTA iteration of the reconstruction at the paper's grid
(128^3 incl. 8-cell PML, 128x128 sensor plane, Nt = 740, CFL 0.3): A^T C^T of
the extrapolated residual, the gradient step, the positivity-constrained TV
prox (50 PDHG iterations, Dirichlet TV), A and C of the new iterate, the FP64
energy/residual/TV/PSNR reductions and the FISTA extrapolation in image and
data space, with restart + backtracking enabled; the call ends with the
Bregman update. value = forward/adjoint pairs executed per second (one pair
per iteration plus the pairs of any restart; the loop starts from p = 0, whose
residual -f needs no operator application).

Inputs are synthetic and already resident in HBM: 24 random vessels (radius
1-4 voxels), random 12.5 % single points (2048 of 16384 pixels, default) or
2048 scrambled Hadamard patterns (--sampling hadamard), 1 % Gaussian noise.

Prints ONE JSON line on stdout; progress goes to stderr.
"""

import argparse
import hashlib
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "fwd+adj operator pairs/s at 128^3; time-to-target-PSNR vs plain TV-Bregman"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def code_only(text):
    """Source text without comments and blank lines (comment edits keep the hash)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*", "", ln).strip() for ln in text.splitlines())
    return "\n".join(ln for ln in lines if ln)


def kernel_source_hash(read=None):
    """Hash of the propagator kernel sources (code only)."""
    h = hashlib.sha256()
    for f in ("line_kernels.hip", "line_common.hpp", "kspace.hpp", "wave_kernels.hip", "fft_radix.hpp",
              "wave_common.hpp"):
        path = os.path.join(ROOT, "paper_1605_00133_amd", "csrc", f)
        text = read(f) if read else open(path, encoding="utf-8").read()
        h.update(code_only(text).encode())
    return h.hexdigest()[:16]


def measured_traffic(kernel_name, src_hash):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if the kernel is unchanged."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(kernel_name)
    except (ValueError, OSError):
        return None
    if not rec or rec.get("source_hash") != src_hash:
        return None
    return rec.get("bytes_per_launch")


def cpu_baseline(n, nt, p0, smp_kind, mc, idx, perm, steps):
    """The FP64 oracle on the host, `steps` forward and `steps` adjoint time steps, scaled to one pair."""
    import oracle
    from oracle.sampling import Sampling, apply_c, apply_ct
    cores = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    cores = max(1, min(cores, os.cpu_count() or 1))
    g = oracle.Grid(n, n, n, dx=100e-6, c0=1500.0, dt=20e-9, nt=steps + 1, pml_size=8)
    op = oracle.WaveOperator(g, workers=cores)
    smp = Sampling(smp_kind, mc, idx=idx, perm=perm) if smp_kind != "full" else Sampling.full(n * n)
    t0 = time.perf_counter()
    f = apply_c(op.forward_planes(p0), smp)
    op.adjoint_planes(apply_ct(f, smp, n, n))
    dt = time.perf_counter() - t0
    pair_s = dt * (nt - 1) / steps
    return {"value": 1.0 / pair_s, "unit": "pairs/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} forward + {steps} adjoint time steps of the FP64 NumPy oracle at {n}^3 "
                      f"({dt:.1f} s), scaled by {nt - 1}/{steps} to one pair"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--sampling", choices=["points", "hadamard"], default="points")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--nt", type=int, default=740)
    ap.add_argument("--n-prox", type=int, default=50)
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--scheme", choices=["line", "slab"], default="line",
                    help="propagator implementation (line needs FP64 butterflies)")
    ap.add_argument("--fft-precision", type=int, choices=[32, 64], default=64,
                    help="arithmetic of the FFT butterflies (storage is FP32 either way)")
    ap.add_argument("--concurrent", type=int, default=2,
                    help="also time this many independent problems at once, one plan and stream each "
                         "(reported apart from the value; 0 or 1: skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the hot path has no multi-GPU mode "
              "(independent problems shard trivially, see DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1605_00133_amd import pat as P
    from synthetic import gaussian_data, gaussian_volume, vessel_phantom

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    n, nt, pml = args.n, args.nt, 8
    npix, mc = n * n, (n * n) // 8
    if args.sampling == "points":
        idx, perm = P.pat_make_rsp_mask(npix, mc, 2), None
    else:
        perm, idx = P.pat_make_shd_pattern(npix, mc, 4)
    grid = P.make_grid(n, n, n, 100e-6, 1500.0, 20e-9, nt, pml)
    plan = P.Plan(grid, args.sampling, mc, idx, perm)
    plan.set_fft_precision(args.fft_precision)
    if args.fft_precision == 64:
        plan.set_scheme(args.scheme)
    log(f"plan {n}^3 nt={nt} {args.sampling} mc={mc}: workspace {plan.workspace.numel() / 2**20:.0f} MiB")

    p0_h = vessel_phantom((n, n, n), pml, 24, 1.0, 4.0, 1)
    p0 = torch.from_numpy(p0_h.astype(np.float32)).to(dev)
    f = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
    P.pat_forward(plan, p0, f)
    torch.cuda.synchronize()
    sigma = 0.01 * float(f.abs().max())
    f += sigma * torch.from_numpy(gaussian_data(plan.data_shape, 3).astype(np.float32)).to(dev)
    x0 = torch.from_numpy(gaussian_volume(plan.vol_shape, 8).astype(np.float32)).to(dev)
    L = P.pat_power_iteration(plan, x0, 10)
    lam = 2e-3 * sigma * np.sqrt(nt * mc) / 1.0
    log(f"L = {L:.4e}, sigma = {sigma:.3e}, lambda = {lam:.3e}")
    p = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)

    def run(iters):
        return P.pat_reconstruct(plan, f, p, lam, L, n_outer=1, n_inner=iters, n_prox=args.n_prox,
                                 bc="dirichlet", restart=True, p_ref=p0)

    if args.warmup > 0:
        run(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = run(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    flags = out["flags"]
    n_fwd = args.steps + int(flags.sum())
    n_adj = args.steps + int((flags > 0).sum())
    pairs = 0.5 * (n_fwd + n_adj)
    elapsed = t1 - t0
    log(f"timed: {args.steps} FISTA steps in {elapsed:.3f} s, {pairs} pairs, restarts {int((flags > 0).sum())}, "
        f"final PSNR {out['psnr'][-1]:.2f} dB")

    # operator-only pairs (A then A^T, nothing else)
    g = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)
    ftmp = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(3):
        P.pat_forward(plan, p0, ftmp)
        P.pat_adjoint(plan, ftmp, g)
    torch.cuda.synchronize()
    op_pairs_s = 3 / (time.perf_counter() - t2)

    # live per-kernel timing of one pair with HIP events on the plan's stream
    P.pat_profile_begin(plan, -2, 8 * nt + 64)
    P.pat_forward(plan, p0, ftmp)
    P.pat_adjoint(plan, ftmp, g)
    tot_ms, launches = P.pat_profile_end(plan)
    kernels = {}
    for k in range(P.PAT_K_COUNT):
        if launches[k] == 0:   # kernels of the scheme that is not running
            continue
        name, nbytes = P.pat_kernel_info(plan, k)
        avg = tot_ms[k] / max(1, launches[k])
        kernels[name] = {"avg_us": round(avg * 1e3, 3), "launches": int(launches[k]),
                         "total_ms": round(float(tot_ms[k]), 3),
                         "GBps": round(nbytes / (avg * 1e-3) / 1e9, 1) if avg > 0 else None,
                         "alg_bytes": nbytes}
    dom = max(kernels, key=lambda k: kernels[k]["total_ms"])
    dk = kernels[dom]
    src_hash = kernel_source_hash()
    traffic = measured_traffic(dom, src_hash)
    roofline = {"bound": "hbm", "achieved": dk["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dk["GBps"] / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "alg_bytes_per_launch": dk["alg_bytes"], "avg_launch_us": dk["avg_us"]}

    # independent problems (other phantoms, parameter sweeps, frames of a 4D scan)
    # overlap on the GPU when each has its own plan and stream: aggregate rate
    concurrent = None
    if args.concurrent > 1:
        K = args.concurrent
        plans = [plan] + [P.Plan(grid, args.sampling, mc, idx, perm) for _ in range(K - 1)]
        for q in plans[1:]:
            q.set_fft_precision(args.fft_precision)
            if args.fft_precision == 64:
                q.set_scheme(args.scheme)
        streams = [torch.cuda.Stream(device=dev) for _ in range(K)]   # default priority
        xs = [torch.from_numpy(vessel_phantom((n, n, n), pml, 24, 1.0, 4.0, 1 + k).astype(np.float32)).to(dev)
              for k in range(K)]
        fk = [torch.empty(plan.data_shape, dtype=torch.float32, device=dev) for _ in range(K)]
        gk = [torch.empty(plan.vol_shape, dtype=torch.float32, device=dev) for _ in range(K)]

        def run_all():
            for k in range(K):
                with torch.cuda.stream(streams[k]):
                    P.pat_forward(plans[k], xs[k], fk[k])
                    P.pat_adjoint(plans[k], fk[k], gk[k])

        torch.cuda.synchronize()
        run_all()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        for _ in range(2):
            run_all()
        torch.cuda.synchronize()
        agg = 2 * K / (time.perf_counter() - t3)
        concurrent = {"problems": K, "aggregate_operator_pairs_per_s": round(agg, 4),
                      "vs_single": round(agg / op_pairs_s, 3),
                      "note": f"independent {n}^3 problems, one plan and stream each; not the value"}
        log(f"concurrent: {K} problems, {agg:.2f} operator pairs/s aggregate ({agg / op_pairs_s:.2f}x one)")
        for q in plans[1:]:
            q.close()

    cpu = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle {args.cpu_steps}+{args.cpu_steps} steps at {n}^3 ...")
        cpu = cpu_baseline(n, nt, p0_h, args.sampling, mc, np.asarray(idx), None if perm is None else np.asarray(perm),
                           args.cpu_steps)

    res = {
        "metric": METRIC, "value": round(pairs / elapsed, 4), "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "fft_arithmetic": f"f{args.fft_precision}",
        "scheme": args.scheme if args.fft_precision == 64 else "slab",
        "data": "synthetic (random vessel phantom, seeded mask, 1% Gaussian noise)",
        "config": {"workload": f"{n}^3 grid incl. 8-cell PML, Nt={nt}, {args.sampling} sampling mc={mc}, "
                               f"one TV FISTA iteration per step ({args.n_prox} PDHG, restart on) inside TV+Br",
                   "grid": n, "nt": nt, "sampling": args.sampling, "mc": mc, "n_prox": args.n_prox,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "operator_pairs_per_s": round(op_pairs_s, 4),
        "concurrent": concurrent,
        "kernels": kernels,
        "kernel_source_hash": src_hash,
        "final_psnr_db": round(float(out["psnr"][-1]), 3),
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
