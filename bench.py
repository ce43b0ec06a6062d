"""Benchmark: fwd+adj operator pairs/s at 128^3 inside TV-Bregman FISTA, and the
time to target PSNR of plain TV-Bregman.

Workload (paper_1605_00133_amd.workload): the paper's grid (128^3 incl. 8-cell
PML, 128x128 detection plane, Nt = 740, CFL 0.3), 24 random vessels (radius 1-4
voxels), random 12.5 % single points (2048 of 16384 pixels, default) or 2048
scrambled Hadamard patterns (--sampling hadamard), 1 % Gaussian noise;
lambda_Br = 10 lambda_TV+, lambda_TV+ fixed beforehand by the discrepancy
principle (eq. DiscPr) and frozen in synthetic.CONFIGS.

A step is one FISTA iteration of the first TV+Br outer step: A^T C^T of the
extrapolated residual, the gradient step, the positivity-constrained TV prox
(50 PDHG iterations, Dirichlet TV), A and C of the new iterate, the FP64
energy/residual/TV/PSNR reductions and the extrapolation in image and data
space, with restart + backtracking on. value = forward/adjoint pairs executed
per second (one pair per iteration plus the pairs of any restart; the loop
starts from p = 0, whose residual -f needs no operator application).

Besides the value (all outside the timed region): operator-only pairs/s; the
per-kernel HIP-event timing of one pair (roofline of the dominant kernel); the
error of this run's A and A^T against stored FP64 oracle samples; the other
sampling mode's rates; 2 and 4 independent problems at once (4 x 0.5 GB is
above the 256 MB last-level cache); with patterned interrogation (the learned
update's workload) the time-to-target curve of plain TV+Br (5 x 50, PSNR and
wall time per iteration) and, when trained weights are present, the learned
reconstruction against it, on this phantom and on held-out phantoms 5004...
(--learned-phantoms) against their own TV+Br runs; the FP64 oracle timed on the
host (all cores and one core).

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
GOLDEN = os.path.join(ROOT, "tests", "golden")


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


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def fp64_error(P, torch, prob):
    """Relative L2 error of this run's A and A^T against the FP64 oracle samples stored
    by tests/golden/make_operator_fixtures.py (None where the fixture is absent)."""
    from synthetic import gaussian_data
    kind, plan, dev = prob["sampling"], prob["plan"], prob["f"].device
    out = {}
    path = os.path.join(GOLDEN, f"op128_forward_{kind}.npz")
    if prob["n"] == 128 and prob["nt"] == 740 and os.path.exists(path):
        fx = np.load(path)
        f = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
        P.pat_forward(plan, prob["p0"], f)
        fh = f.cpu().numpy().astype(np.float64)
        out["forward_sampled_columns"] = rel_l2(fh[:, fx["cols"]], fx["values"])
        out["forward_norm"] = abs(np.linalg.norm(fh) - float(fx["norm"])) / float(fx["norm"])
    path = os.path.join(GOLDEN, f"op128_adjoint_{kind}.npz")
    if prob["n"] == 128 and prob["nt"] == 740 and os.path.exists(path):
        fx = np.load(path)
        y = torch.from_numpy(gaussian_data(plan.data_shape, int(fx["data_seed"])).astype(np.float32)).to(dev)
        p = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)
        P.pat_adjoint(plan, y, p)
        ph = p.cpu().numpy().astype(np.float64)
        out["adjoint_sampled_slices"] = rel_l2(ph[fx["zs"]], fx["values"])
        out["adjoint_norm"] = abs(np.linalg.norm(ph) - float(fx["norm"])) / float(fx["norm"])
    return out or None


def ensure_lambda(prob):
    """A grid other than the frozen workload's has no calibrated lambda: the frozen fraction of
    sigma sqrt(Nt M_c) of the random-point calibration stands in."""
    if prob["lam_br"] is None:
        prob["lam_tv"] = 6.3e-4 * prob["sigma"] * np.sqrt(prob["plan"].data_shape[0] * prob["mc"])
        prob["lam_br"] = 10.0 * prob["lam_tv"]
    return prob


def fista_rate(P, torch, prob, steps, warmup, n_prox):
    """`steps` FISTA iterations of the first TV+Br outer step, timed; returns (pairs, seconds, log)."""
    plan, f = prob["plan"], prob["f"]
    p = torch.empty(plan.vol_shape, dtype=torch.float32, device=f.device)

    def run(iters):
        return P.pat_reconstruct(plan, f, p, prob["lam_br"], prob["L"], n_outer=1, n_inner=iters, n_prox=n_prox,
                                 bc="dirichlet", restart=True, p_ref=prob["p0"])

    if warmup > 0:
        run(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = run(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    flags = out["flags"]
    n_fwd = steps + int(flags.sum())
    n_adj = steps + int((flags > 0).sum())
    return 0.5 * (n_fwd + n_adj), elapsed, out


def operator_rate(P, torch, prob, pairs=10, per_pair=None):
    """Operator-only pairs/s over `pairs` back-to-back pairs (host clock); with a dict per_pair,
    also each pair's duration by HIP events on the current stream (median, min ms)."""
    plan, dev = prob["plan"], prob["f"].device
    g = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)
    ftmp = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
    P.pat_forward(plan, prob["p0"], ftmp)
    P.pat_adjoint(plan, ftmp, g)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(pairs + 1)]
    torch.cuda.synchronize()
    t = time.perf_counter()
    ev[0].record()
    for i in range(pairs):
        P.pat_forward(plan, prob["p0"], ftmp)
        P.pat_adjoint(plan, ftmp, g)
        ev[i + 1].record()
    torch.cuda.synchronize()
    rate = pairs / (time.perf_counter() - t)
    if per_pair is not None:
        ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(pairs))
        per_pair.update({"pairs": pairs, "median_ms": round(float(np.median(ms)), 3), "min_ms": round(ms[0], 3),
                         "max_ms": round(ms[-1], 3)})
    return rate


def copy_ceiling(P, torch, nbytes=1 << 30, reps=5):
    """Device-to-device copy rates (read + write bytes per second, GB/s) of an nbytes buffer: torch's
    copy and the library's copy kernel (pat_copy_probe), median of reps timed copies each;
    the larger is the practical HBM ceiling of this GPU. Returns {"torch": .., "pat_copy_probe": ..}."""
    src = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    src.fill_(1.0)
    dst = torch.empty_like(src)
    rates = {}
    for name, fn in (("torch", lambda: dst.copy_(src)), ("pat_copy_probe", lambda: P.pat_copy_probe(src, dst))):
        fn()
        out = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            torch.cuda.synchronize()
            out.append(2.0 * nbytes / (a.elapsed_time(b) * 1e-3) / 1e9)
        rates[name] = round(float(np.median(out)), 1)
    if not torch.equal(src, dst):
        raise RuntimeError("copy probe: destination differs from source")
    del src, dst
    return rates


def concurrent_rate(P, torch, prob, K, reps=2):
    """Aggregate operator pairs/s of K independent problems (own plan, phantom, stream)."""
    from synthetic import vessel_phantom
    dev = prob["f"].device
    n, grid = prob["n"], prob["plan"].grid
    plans = [P.Plan(grid, prob["sampling"], prob["mc"], prob["idx"], prob["perm"]) for _ in range(K)]
    streams = [torch.cuda.Stream(device=dev) for _ in range(K)]   # default priority
    xs = [torch.from_numpy(vessel_phantom((n, n, n), 8, 24, 1.0, 4.0, 1 + k).astype(np.float32)).to(dev)
          for k in range(K)]
    fk = [torch.empty(plans[0].data_shape, dtype=torch.float32, device=dev) for _ in range(K)]
    gk = [torch.empty(plans[0].vol_shape, dtype=torch.float32, device=dev) for _ in range(K)]

    def run_all():
        for k in range(K):
            with torch.cuda.stream(streams[k]):
                P.pat_forward(plans[k], xs[k], fk[k])
                P.pat_adjoint(plans[k], fk[k], gk[k])

    torch.cuda.synchronize()
    run_all()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        run_all()
    torch.cuda.synchronize()
    agg = reps * K / (time.perf_counter() - t)
    ws = sum(pl.workspace.numel() for pl in plans)
    for pl in plans:
        pl.close()
    return agg, ws


def cpu_baseline(n, nt, p0, smp_kind, mc, idx, perm, steps, workers):
    """The FP64 oracle on the host, `steps` forward and `steps` adjoint time steps, scaled to one pair."""
    import oracle
    from oracle.sampling import Sampling, apply_c, apply_ct
    g = oracle.Grid(n, n, n, dx=100e-6, c0=1500.0, dt=20e-9, nt=steps + 1, pml_size=8)
    op = oracle.WaveOperator(g, workers=workers)
    smp = Sampling(smp_kind, mc, idx=idx, perm=perm) if smp_kind != "full" else Sampling.full(n * n)
    t0 = time.perf_counter()
    f = apply_c(op.forward_planes(p0), smp)
    op.adjoint_planes(apply_ct(f, smp, n, n))
    dt = time.perf_counter() - t0
    pair_s = dt * (nt - 1) / steps
    return {"value": 1.0 / pair_s, "unit": "pairs/s", "cores": workers, "kind": "oracle",
            "sample": f"{steps} forward + {steps} adjoint time steps of the FP64 NumPy oracle at {n}^3 "
                      f"({dt:.1f} s, {workers} FFT thread(s)), scaled by {nt - 1}/{steps} to one pair (extrapolated)"}


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
    ap.add_argument("--cpu-steps-1", type=int, default=3, help="time steps of the one-thread oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-time-to-target", action="store_true")
    ap.add_argument("--learned-phantoms", type=int, default=3,
                    help="held-out phantoms (seeds 5004...) the learned reconstruction is also compared on")
    ap.add_argument("--other-sampling", type=int, default=1, help="also time the other sampling mode (0: skip)")
    ap.add_argument("--concurrent", default="2,4",
                    help="comma-separated counts of independent problems timed at once ('' or 0: skip)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the hot path has no multi-GPU mode (independent problems "
              "such as the frames of a scan would go one per GPU); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1605_00133_amd import pat as P
    from paper_1605_00133_amd.workload import paper_problem, tv_bregman_curve

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n, nt = args.n, args.nt
    prob = ensure_lambda(paper_problem(args.sampling, n, nt))
    plan, mc = prob["plan"], prob["mc"]
    log(f"plan {n}^3 nt={nt} {args.sampling} mc={mc}: workspace {plan.workspace.numel() / 2**20:.0f} MiB; "
        f"L = {prob['L']:.4e}, sigma = {prob['sigma']:.3e}, lambda_TV+ = {prob['lam_tv']:.4e}, "
        f"lambda_Br = {prob['lam_br']:.4e}")

    # ---- the timed region: K FISTA iterations -------------------------------------------
    pairs, elapsed, out = fista_rate(P, torch, prob, args.steps, args.warmup, args.n_prox)
    flags = out["flags"]
    log(f"timed: {args.steps} FISTA steps in {elapsed:.3f} s, {pairs} pairs, restarts {int((flags > 0).sum())}, "
        f"PSNR after them {out['psnr'][-1]:.2f} dB")

    pair_ms = {}
    op_pairs_s = operator_rate(P, torch, prob, per_pair=pair_ms)
    copy_rates = copy_ceiling(P, torch)
    copy_GBps = max(copy_rates.values())
    log(f"operator pairs: {op_pairs_s:.2f}/s, per pair median {pair_ms['median_ms']:.2f} ms (min {pair_ms['min_ms']:.2f}); "
        f"device copy: torch {copy_rates['torch']:.0f} GB/s, pat_copy_probe {copy_rates['pat_copy_probe']:.0f} GB/s")

    # ---- live per-kernel timing of one pair with HIP events on the plan's stream ----------
    dev = prob["f"].device
    g = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)
    ftmp = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
    P.pat_profile_begin(plan, -2, 8 * nt + 64)
    P.pat_forward(plan, prob["p0"], ftmp)
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
    R, Cb = 4.0 * n ** 3, 8.0 * n * n * (n // 2 + 1)
    fft_step_bytes = 20 * Cb + 12 * R     # one time step at two global passes per 3D FFT
    roofline = {"bound": "hbm", "achieved": dk["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(dk["GBps"] / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": dom,
                "alg_bytes_per_launch": dk["alg_bytes"], "avg_launch_us": dk["avg_us"],
                "frac_of_3d_fft_step_bytes": round(fft_step_bytes / (dk["avg_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                "frac_of_copy_ceiling": round(dk["GBps"] / copy_GBps, 4)}

    err = fp64_error(P, torch, prob)
    if err:
        log("error vs FP64 oracle samples: " + ", ".join(f"{k} {v:.2e}" for k, v in err.items()))

    # ---- the other sampling mode --------------------------------------------------------------
    other = None
    if args.other_sampling:
        kind = "hadamard" if args.sampling == "points" else "points"
        prob2 = ensure_lambda(paper_problem(kind, n, nt))
        pr2, el2, _ = fista_rate(P, torch, prob2, max(2, args.steps // 2), 1, args.n_prox)
        other = {"sampling": kind, "fista_pairs_per_s": round(pr2 / el2, 4),
                 "operator_pairs_per_s": round(operator_rate(P, torch, prob2), 4),
                 "fp64_error": fp64_error(P, torch, prob2), "lam_tv": prob2["lam_tv"]}
        log(f"{kind}: {other['fista_pairs_per_s']:.2f} pairs/s in FISTA, {other['operator_pairs_per_s']:.2f} "
            f"operator pairs/s")

    # ---- independent problems at once (above the last-level cache at 4) -----------------------
    concurrent = []
    for K in [int(c) for c in str(args.concurrent).split(",") if c.strip() and int(c) > 1]:
        agg, ws = concurrent_rate(P, torch, prob, K)
        concurrent.append({"problems": K, "aggregate_operator_pairs_per_s": round(agg, 4),
                           "vs_single": round(agg / op_pairs_s, 3), "workspace_bytes": int(ws),
                           "aggregate_alg_GBps": round(agg * 2 * (nt - 1) * dk["alg_bytes"] / 1e9, 1)})
        log(f"concurrent: {K} problems, {agg:.2f} operator pairs/s aggregate ({agg / op_pairs_s:.2f}x one), "
            f"workspaces {ws / 2**20:.0f} MiB")

    # ---- time to target PSNR (patterned interrogation, the learned update's workload): plain TV+Br,
    # and the learned iteration if trained weights are present ----------------------------------
    ttt = None
    if not args.no_time_to_target:
        if args.sampling == "hadamard":
            prob_t = prob
        elif other is not None:
            prob_t = prob2
        else:
            prob_t = ensure_lambda(paper_problem("hadamard", n, nt))
        c = tv_bregman_curve(prob_t, n_prox=args.n_prox)
        ttt = {"sampling": prob_t["sampling"], "lambda_br": prob_t["lam_br"],
               "tv_bregman": {k: v for k, v in c.items() if k not in ("p", "psnr", "t_ms")}}
        ttt["tv_bregman"]["psnr_every_10"] = [round(float(x), 3) for x in c["psnr"][9::10]]
        ttt["tv_bregman"]["t_ms_every_10"] = [round(float(x), 1) for x in c["t_ms"][9::10]]
        log(f"TV+Br 5x50: final {c['final_psnr_db']:.2f} dB after {c['total_ms'] / 1e3:.2f} s; within 0.5 dB "
            f"({c['target_psnr_db']:.2f} dB) at {c['t_target_ms']:.0f} ms (iteration {c['target_iteration']})")
        try:
            from paper_1605_00133_amd.learned_unet import bench_learned
            seeds = tuple(5004 + i for i in range(max(0, args.learned_phantoms)))
            ttt["learned"] = bench_learned(prob_t, c, log=log, extra_seeds=seeds)
        except (ImportError, FileNotFoundError) as e:
            ttt["learned"] = None
            log(f"learned: not run ({e})")

    if other is not None:
        prob2["plan"].close()

    cpu = None
    if not args.no_cpu_baseline:
        import oracle.operator as oop
        cores = oop._workers()
        log(f"cpu baseline: oracle {args.cpu_steps}+{args.cpu_steps} steps at {n}^3 on {cores} threads, "
            f"{args.cpu_steps_1}+{args.cpu_steps_1} on one ...")
        idx, perm = np.asarray(prob["idx"]), None if prob["perm"] is None else np.asarray(prob["perm"])
        cpu = cpu_baseline(n, nt, prob["p0_host"], args.sampling, mc, idx, perm, args.cpu_steps, cores)
        one = cpu_baseline(n, nt, prob["p0_host"], args.sampling, mc, idx, perm, args.cpu_steps_1, 1)
        cpu["single_thread"] = {"value": one["value"], "unit": "pairs/s", "cores": 1, "sample": one["sample"]}

    res = {
        "metric": METRIC, "value": round(pairs / elapsed, 4), "unit": "pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * elapsed / args.steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "fft_arithmetic": "f64", "scheme": "line",
        "data": "synthetic (random vessel phantom, seeded mask, 1% Gaussian noise)",
        "config": {"workload": f"{n}^3 grid incl. 8-cell PML, Nt={nt}, {args.sampling} sampling mc={mc}, "
                               f"one FISTA iteration per step ({args.n_prox} PDHG, restart on) of the first "
                               f"TV+Br outer step, lambda_Br = 10 lambda_TV+ (discrepancy principle)",
                   "grid": n, "nt": nt, "sampling": args.sampling, "mc": mc, "n_prox": args.n_prox,
                   "lambda_tv": prob["lam_tv"], "lambda_br": prob["lam_br"], "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "operator_pairs_per_s": round(op_pairs_s, 4), "operator_pair_ms": pair_ms,
        "copy_ceiling_GBps": round(copy_GBps, 1), "copy_rates_GBps": copy_rates,
        "fp64_error": err,
        "other_sampling": other,
        "concurrent": concurrent,
        "time_to_target": ttt,
        "kernels": kernels,
        "kernel_source_hash": src_hash,
        "psnr_after_timed_steps_db": round(float(out["psnr"][-1]), 3),
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
