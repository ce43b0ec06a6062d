"""Learned reconstruction with U-Net corrections (not part of the paper's method),
trained on and judged by the plain TV-Bregman solver.

K unrolled steps from p_0 = 0, each with a U-Net of its own (paper_1605_00133_amd.unet):
    z_k     = p_k - eta A^T C^T (C A p_k - f)         gradient step, eta = 1.8 / L (eq. BP, App. B)
    p_{k+1} = max(0, z_k + net_k([p_k, z_k]))
The nets are trained one step after another (greedy): z_k + net_k([p_k, z_k])
(before the clamp) is fitted to the plain TV+Br reconstructions of the same data
in mean squared error (Adam), then the next step starts from its clamped outputs.

Fallback: after the K steps the data residual ||C A p_K - f|| (FP64) is compared
with that of plain TV+ FISTA run for the same number of operator pairs (K); if
the learned residual is larger, the plain solver's full TV+Br reconstruction is
returned instead, so the plain solver stays both the fallback and the judge of
the learned result.

Workload (config of the learned update): the paper-scale grid (128^3, Nt = 740)
with 12.5 % scrambled-Hadamard sub-sampling (2048 of 16384 patterns, seeds
4/5), phantoms of 24 random vessels (training seeds 1000 + i, or a later block of
seeds when training continues from saved weights; held-out 5000 + j,
the benchmark phantom 1), 1 % Gaussian noise, TV+Br targets with
lambda_Br = 10 lambda_TV+, lambda_TV+ = lam_tv_rel sigma sqrt(Nt M_c) (the
discrepancy-principle calibration of synthetic.CONFIGS["paper"] scaled to each
phantom's noise level), 5 x 50 FISTA iterations, 50 PDHG steps.

The committed weights (weights/unet_n128_hadamard_w16-32-64.safetensors, 8 steps)
came from three runs of 24 phantoms each:
    --steps 10 --epochs 90 --lr 1e-3                               (seeds 1000-1023)
    --init <that> --train-seed0 1024 --epochs 70 --lr 5e-4          (seeds 1024-1047)
    --init <that> --train-seed0 1048 --steps 8 --epochs 30 --lr 2e-4 (seeds 1048-1071)

Every operation of the learned iteration and of its training runs in libpat:
pat_forward / pat_adjoint, pat_axpby, the U-Net's convolution, resampling and
add kernels, pat_mse and pat_adam_step. Weights are saved with safetensors
(convolution weights as bfloat16, the precision the matrix cores multiply in;
biases as float32).
"""

import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import nn
from . import pat as P
from .unet import UNet

PKG = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_DIR = os.path.join(PKG, "weights")


def weights_path(n, sampling, widths=(16, 32, 64)):
    return os.path.join(WEIGHTS_DIR, f"unet_n{n}_{sampling}_w{'-'.join(str(w) for w in widths)}.safetensors")


def gradient_step(plan, f, p, eta, r=None, g=None):
    """z = p - eta A^T C^T (C A p - f) for one volume [nz, ny, nx]; r, g: optional scratch tensors."""
    r = torch.empty(plan.data_shape, dtype=torch.float32, device=p.device) if r is None else r
    g = torch.empty(plan.vol_shape, dtype=torch.float32, device=p.device) if g is None else g
    P.pat_forward(plan, p, r)
    nn.axpby(r, f, 1.0, -1.0, out=r)
    P.pat_adjoint(plan, r, g)
    return nn.axpby(p, g, 1.0, -eta)


def residual_norm(plan, f, p):
    """||C A p - f|| with an FP64 reduction (host float; syncs)."""
    r = torch.empty(plan.data_shape, dtype=torch.float32, device=p.device)
    P.pat_forward(plan, p, r)
    return math.sqrt(float(nn.mse(r, f)) * r.numel())


class LearnedUNetRecon:
    """K unrolled steps with a U-Net each."""

    def __init__(self, n_steps=8, widths=(16, 32, 64), seed=0, device="cuda:0"):
        self.widths = tuple(widths)
        self.nets = [UNet(widths, seed + 17 * k, device) for k in range(n_steps)]

    @property
    def n_steps(self):
        return len(self.nets)

    def truncated(self, k):
        """The first k steps (greedy training makes them the k-step model)."""
        if not 1 <= k <= self.n_steps:
            raise ValueError(f"k must be in [1, {self.n_steps}]")
        out = LearnedUNetRecon.__new__(LearnedUNetRecon)
        out.widths, out.nets = self.widths, self.nets[:k]
        return out

    @property
    def n_params(self):
        return sum(net.n_params for net in self.nets)

    def step(self, k, p, z, keep=False, clamp=True):
        """p_{k+1} = max(0, z + net_k([p, z])) for [B, 1, N, N, N] tensors p, z (clamp=False: the
        value before the clamp, which training fits: through the clamp a step whose output has
        gone negative everywhere gets no gradient and cannot recover)."""
        x = torch.empty((p.shape[0], 2) + tuple(p.shape[2:]), dtype=torch.float32, device=p.device)
        for b in range(p.shape[0]):
            nn.axpby(p[b, 0], None, 1.0, out=x[b, 0])
            nn.axpby(z[b, 0], None, 1.0, out=x[b, 1])
        out = self.nets[k].forward(x, keep=keep)
        return nn.axpby(z, out, 1.0, 1.0, clamp0=clamp)

    def reconstruct(self, plan, f, L):
        """p_K for data f [Nt, M_c]; K operator pairs and K U-Net evaluations."""
        eta = 1.8 / L
        p = torch.zeros(plan.vol_shape, dtype=torch.float32, device=f.device)
        r = torch.empty(plan.data_shape, dtype=torch.float32, device=f.device)
        g = torch.empty(plan.vol_shape, dtype=torch.float32, device=f.device)
        for k in range(self.n_steps):
            z = gradient_step(plan, f, p, eta, r, g)
            p = self.step(k, p[None, None], z[None, None])[0, 0]
        return p

    def save(self, path):
        from safetensors.torch import save_file
        sd = {}
        for k, net in enumerate(self.nets):
            for name, t in net.state_dict().items():
                sd[f"step{k}.{name}"] = t.to(torch.bfloat16) if name.endswith(".0") else t.float()
        os.makedirs(os.path.dirname(path), exist_ok=True)
        save_file(sd, path, metadata={"widths": json.dumps(list(self.widths)), "n_steps": str(self.n_steps)})

    @classmethod
    def load(cls, path, device="cuda:0"):
        from safetensors import safe_open
        from safetensors.torch import load_file
        with safe_open(path, framework="pt") as fh:
            meta = fh.metadata()
        model = cls(int(meta["n_steps"]), tuple(json.loads(meta["widths"])), 0, device)
        sd = load_file(path)
        for k, net in enumerate(model.nets):
            net.load_state_dict({name[len(f"step{k}."):]: t for name, t in sd.items() if name.startswith(f"step{k}.")})
        return model


def reconstruct_with_fallback(model, plan, f, L, lam_tv, lam_br, n_prox=50, p_ref=None, ref_plan=None):
    """The learned reconstruction, or plain TV+Br when its data residual is larger than that of plain
    TV+ FISTA (no restart) with the same number of operator pairs. With `ref_plan` (a second plan of
    the same grid and sampling) that reference runs on a stream of its own, concurrently with the
    learned steps; without it, after them. Returns (p, info)."""
    dev = f.device
    t0 = time.perf_counter()
    q = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)
    log = torch.zeros((model.n_steps, 2), dtype=torch.float64, device=dev)
    cur = torch.cuda.current_stream(dev)
    if ref_plan is not None:
        side = torch.cuda.Stream(device=dev)      # default priority
        side.wait_stream(cur)
        with torch.cuda.stream(side):
            P.pat_fista_enqueue(ref_plan, f, q, lam_tv, L, model.n_steps, n_prox, "dirichlet", log)
        p = model.reconstruct(plan, f, L)         # on the caller's stream, concurrently
        r_learned = residual_norm(plan, f, p)
        cur.wait_stream(side)
        ref_plan.sync_stream()
    else:
        p = model.reconstruct(plan, f, L)
        r_learned = residual_norm(plan, f, p)
        P.pat_fista_enqueue(plan, f, q, lam_tv, L, model.n_steps, n_prox, "dirichlet", log)
    r_plain = math.sqrt(float(log[-1, 0]))
    fallback = not (r_learned <= r_plain)
    if fallback:
        P.pat_reconstruct(plan, f, q, lam_br, L, n_outer=5, n_inner=50, n_prox=n_prox, bc="dirichlet", restart=True)
        p = q
    torch.cuda.synchronize(dev)
    info = {"residual_learned": r_learned, "residual_plain_same_pairs": r_plain, "fallback": fallback,
            "ms": 1e3 * (time.perf_counter() - t0), "concurrent_reference": ref_plan is not None}
    if p_ref is not None:
        info["psnr_db"] = P.pat_psnr(plan, p, p_ref)
    return p, info


# ---- data, targets and training -----------------------------------------------------------
def make_plan(n=128, sampling="hadamard", device="cuda:0"):
    from synthetic import CONFIGS
    cfg = CONFIGS["paper"]
    nt = int(round(cfg["nt"] * n / cfg["n"]))
    npix, mc = n * n, n * n // 8
    if sampling == "hadamard":
        perm, idx = P.pat_make_shd_pattern(npix, mc, cfg["hadamard_seed"])
    else:
        idx, perm = P.pat_make_rsp_mask(npix, mc, cfg["mask_seed"]), None
    grid = P.make_grid(n, n, n, cfg["dx"], cfg["c0"], cfg["dt"], nt, cfg["pml"], cfg["pml_alpha"])
    return P.Plan(grid, sampling, mc, idx, perm, device=device)


def make_case(plan, seed, sampling, device="cuda:0"):
    """Phantom (seed), data with 1 % noise (seed + 1000), sigma and the TV+ / TV+Br weights."""
    from synthetic import CONFIGS, gaussian_data, vessel_phantom
    cfg = CONFIGS["paper"]
    n = plan.grid.nx
    nv, rmax = (cfg["n_vessels"], cfg["r_max"]) if n >= 64 else (6, 2.0)
    p0 = torch.from_numpy(vessel_phantom((n, n, n), cfg["pml"], nv, cfg["r_min"], rmax, seed).astype(np.float32))
    p0 = p0.to(device)
    f = torch.empty(plan.data_shape, dtype=torch.float32, device=device)
    P.pat_forward(plan, p0, f)
    torch.cuda.synchronize(device)
    sigma = cfg["noise_rel"] * float(f.abs().max())
    noise = torch.from_numpy(gaussian_data(plan.data_shape, seed + 1000).astype(np.float32)).to(device)
    nn.axpby(f, noise, 1.0, sigma, out=f)
    lam_tv = cfg["lam_tv_rel"][sampling] * sigma * math.sqrt(plan.data_shape[0] * plan.data_shape[1])
    return {"p0": p0, "f": f, "sigma": sigma, "lam_tv": lam_tv, "lam_br": cfg["br_factor"] * lam_tv, "seed": seed}


def tv_bregman(plan, case, L, n_prox=50, p_ref=None):
    """Plain TV+Br (5 x 50) of a case: (p, log)."""
    p = torch.empty(plan.vol_shape, dtype=torch.float32, device=case["f"].device)
    log = P.pat_reconstruct(plan, case["f"], p, case["lam_br"], L, n_outer=5, n_inner=50, n_prox=n_prox,
                            bc="dirichlet", restart=True, p_ref=p_ref)
    return p, log


def train(model, plan, fs, targets, L, epochs=40, batch=2, lr=1e-3, log=None):
    """Greedy training (see the module docstring), Adam with the rate decaying linearly from lr to
    lr / 10 over each step's updates; returns the final training MSE of each step."""
    eta = 1.8 / L
    n = len(fs)
    dev = fs[0].device
    ps = [torch.zeros((1, 1) + plan.vol_shape, dtype=torch.float32, device=dev) for _ in range(n)]
    losses = []
    gen = torch.Generator().manual_seed(1)
    r = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
    g = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)
    for k in range(model.n_steps):
        zs = [gradient_step(plan, f, p[0, 0], eta, r, g)[None, None] for f, p in zip(fs, ps)]
        net = model.nets[k]
        moments = {name: ([torch.zeros_like(t) for t in wb], [torch.zeros_like(t) for t in wb])
                   for name, wb in net.params.items()}
        t_adam = 0
        total = epochs * ((n + batch - 1) // batch)
        t0 = time.perf_counter()
        for ep in range(epochs):
            perm = torch.randperm(n, generator=gen).tolist()
            for s in range(0, n, batch):
                idx = perm[s:s + batch]
                pb = torch.cat([ps[i] for i in idx])
                zb = torch.cat([zs[i] for i in idx])
                tb = torch.stack([targets[i] for i in idx])[:, None].contiguous()
                out = model.step(k, pb, zb, keep=True, clamp=False)
                dout = torch.empty_like(out)
                nn.mse(out, tb, grad=dout)
                grads = net.backward(dout)
                t_adam += 1
                for name, wb in net.params.items():
                    m, v = moments[name]
                    for i in range(2):
                        nn.adam_step_(wb[i], grads[name][i].contiguous(), m[i], v[i], t_adam,
                                      lr=lr * (1.0 - 0.9 * (t_adam - 1) / total))
        with torch.no_grad():
            ps = [model.step(k, p, z) for p, z in zip(ps, zs)]
            mse = float(np.mean([float(nn.mse(p[0, 0], t)) for p, t in zip(ps, targets)]))
        losses.append(mse)
        if log:
            log(f"step {k}: training MSE {mse:.3e} ({time.perf_counter() - t0:.1f} s)")
    return losses


def initial_model(n_steps, widths, init=None, device="cuda:0"):
    """Fresh nets (seed 0), or the first n_steps nets of the saved model init (same widths)."""
    if not init:
        return LearnedUNetRecon(n_steps, widths, 0, device)
    model = LearnedUNetRecon.load(init, device)
    if model.n_steps < n_steps or model.widths != tuple(widths):
        raise ValueError(f"{init}: {model.n_steps} steps of widths {model.widths}, asked for {n_steps} of "
                         f"{tuple(widths)}")
    return model.truncated(n_steps)


def experiment(n=128, sampling="hadamard", n_train=24, n_test=4, n_steps=8, widths=(16, 32, 64), epochs=40,
               batch=2, lr=1e-3, workers=2, save=None, eval_steps=None, log=None, init=None, train_seed0=1000):
    """Trains on n_train phantoms (seeds train_seed0 + i), evaluates on n_test held-out ones
    (seeds 5000 + j) against plain TV+Br (time to within 0.5 dB of its final PSNR vs the learned
    iteration's time, fallback included). init: a saved model whose first n_steps nets are the
    starting point (training continued on further phantoms) instead of fresh nets."""
    if train_seed0 < 0 or train_seed0 + n_train > 5000:
        raise ValueError("training phantoms must not overlap the held-out seeds 5000 + j")
    dev = torch.device("cuda:0")
    model = initial_model(n_steps, widths, init, dev)
    from synthetic import gaussian_volume
    from .frames import reconstruct_all
    from .workload import target_time
    plan = make_plan(n, sampling)
    x0 = torch.from_numpy(gaussian_volume(plan.vol_shape, 8).astype(np.float32)).to(dev)
    L = P.pat_power_iteration(plan, x0, 10)
    train_cases = [make_case(plan, train_seed0 + i, sampling) for i in range(n_train)]
    test_cases = [make_case(plan, 5000 + j, sampling) for j in range(n_test)]
    t0 = time.perf_counter()
    plans = [plan] + [make_plan(n, sampling) for _ in range(max(0, workers - 1))]
    targets = [torch.empty(plan.vol_shape, dtype=torch.float32, device=dev) for _ in train_cases]
    for c0 in range(0, n_train, len(plans)):
        c1 = min(c0 + len(plans), n_train)
        reconstruct_all(plans[:c1 - c0], [c["f"] for c in train_cases[c0:c1]], targets[c0:c1],
                        [c["lam_br"] for c in train_cases[c0:c1]], [L] * (c1 - c0), workers=len(plans),
                        n_outer=5, n_inner=50, n_prox=50)
        if log:
            log(f"targets {c1}/{n_train} ({time.perf_counter() - t0:.0f} s)")
    for q in plans[1:]:
        q.close()
    torch.cuda.synchronize()
    t_targets = time.perf_counter() - t0
    t0 = time.perf_counter()
    losses = train(model, plan, [c["f"] for c in train_cases], targets, L, epochs=epochs, batch=batch, lr=lr,
                   log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    if save:
        model.save(save)
    del targets
    ks = sorted(set(eval_steps or ()) | {n_steps})
    rows = {k: [] for k in ks}
    ref_plan = make_plan(n, sampling)
    for c in test_cases:
        ref = tv_bregman_reference(plan, c, L)
        for k in ks:
            rows[k].append(evaluate_case(model.truncated(k), plan, c, L, ref, ref_plan))
        if log:
            log(f"case {c['seed']}: TV+Br {ref['tvbr_final_db']:.2f} dB, " + ", ".join(
                f"K={k}: {rows[k][-1]['learned_db']:.2f} dB in {rows[k][-1]['learned_ms']:.0f} ms" for k in ks))
    summary = {}
    for k in ks:
        summary[f"k{k}"] = summarize(rows[k])
        summary[f"k{k}"]["cases"] = rows[k]
        if log:
            log(f"K = {k}: {json.dumps({a: b for a, b in summary[f'k{k}'].items() if a != 'cases'})}")
    summary.update({"n": n, "sampling": sampling, "n_train": n_train, "n_test": n_test, "n_steps": n_steps,
                    "widths": list(widths), "n_params": model.n_params, "epochs": epochs, "batch": batch, "lr": lr,
                    "train_mse": losses, "targets_s": t_targets, "train_s": t_train, "L": L,
                    "train_seed0": train_seed0, "init": os.path.basename(init) if init else None})
    ref_plan.close()
    plan.close()
    return summary


def tv_bregman_reference(plan, case, L):
    """Plain TV+Br (5 x 50) of a case with PSNR logged: its final PSNR and time to within 0.5 dB."""
    from .workload import target_time
    torch.cuda.synchronize()
    _, log = tv_bregman(plan, case, L, p_ref=case["p0"])
    target, t_target, it = target_time(log["psnr"], log["t_ms"])
    return {"tvbr_final_db": float(log["psnr"][-1]), "tvbr_target_db": target, "tvbr_t_target_ms": t_target,
            "tvbr_total_ms": float(log["t_ms"][-1]), "tvbr_target_iteration": it,
            "_psnr": np.asarray(log["psnr"], dtype=np.float64), "_t_ms": np.asarray(log["t_ms"], dtype=np.float64)}


def psnr_at_time(ref, t_ms):
    """PSNR of the plain TV+Br run at wall time t_ms (its last logged iteration by then; -inf before
    the first)."""
    done = np.nonzero(ref["_t_ms"] <= t_ms)[0]
    return float(ref["_psnr"][done[-1]]) if done.size else float("-inf")


def evaluate_case(model, plan, case, L, ref=None, ref_plan=None):
    """The learned reconstruction (with its fallback check) on one case against plain TV+Br."""
    ref = tv_bregman_reference(plan, case, L) if ref is None else ref
    _, info = reconstruct_with_fallback(model, plan, case["f"], L, case["lam_tv"], case["lam_br"], p_ref=case["p0"],
                                        ref_plan=ref_plan)
    row = {"seed": case["seed"], "n_steps": model.n_steps}
    row.update({k: v for k, v in ref.items() if not k.startswith("_")})
    tvbr_same_time = psnr_at_time(ref, info["ms"])
    row.update({"learned_db": info["psnr_db"], "learned_ms": info["ms"], "fallback": info["fallback"],
                "tvbr_db_at_learned_time": tvbr_same_time, "gain_vs_tvbr_same_time": info["psnr_db"] - tvbr_same_time,
                "residual_learned": info["residual_learned"],
                "residual_plain_same_pairs": info["residual_plain_same_pairs"],
                "db_vs_tvbr": info["psnr_db"] - ref["tvbr_final_db"],
                "speedup_vs_target_time": ref["tvbr_t_target_ms"] / info["ms"],
                "speedup_vs_full_tvbr": ref["tvbr_total_ms"] / info["ms"]})
    return row


def summarize(rows):
    keys = ("db_vs_tvbr", "speedup_vs_target_time", "speedup_vs_full_tvbr", "learned_db", "tvbr_final_db",
            "learned_ms", "tvbr_t_target_ms", "gain_vs_tvbr_same_time")
    out = {f"mean_{k}": float(np.mean([r[k] for r in rows])) for k in keys}
    out["min_db_vs_tvbr"] = float(np.min([r["db_vs_tvbr"] for r in rows]))
    out["min_speedup_vs_target_time"] = float(np.min([r["speedup_vs_target_time"] for r in rows]))
    out["fallbacks"] = int(sum(r["fallback"] for r in rows))
    return out


def bench_learned(prob, curve, log=None, n_steps=8, widths=(16, 32, 64), extra_seeds=(5004, 5005, 5006)):
    """The learned iteration (first n_steps steps of the committed weights) on the benchmark's problem
    (a held-out phantom), against the plain TV+Br curve `curve` of the same problem, and on the
    held-out phantoms `extra_seeds` (make_case) against their own TV+Br runs; the means are over all
    of them. Raises FileNotFoundError without weights."""
    path = weights_path(prob["n"], prob["sampling"], widths)
    if not os.path.exists(path):
        raise FileNotFoundError(path)
    model = LearnedUNetRecon.load(path, prob["f"].device)
    model = model.truncated(min(n_steps, model.n_steps))
    plan, f, L = prob["plan"], prob["f"], prob["L"]
    ref_plan = P.Plan(plan.grid, prob["sampling"], prob["mc"], prob["idx"], prob["perm"], device=f.device)
    reconstruct_with_fallback(model, plan, f, L, prob["lam_tv"], prob["lam_br"], ref_plan=ref_plan)   # warm-up
    _, info = reconstruct_with_fallback(model, plan, f, L, prob["lam_tv"], prob["lam_br"], p_ref=prob["p0"],
                                        ref_plan=ref_plan)
    rows = [evaluate_case(model, plan, make_case(plan, seed, prob["sampling"]), L, ref_plan=ref_plan)
            for seed in extra_seeds]
    ref_plan.close()
    out = {"weights": os.path.relpath(path, os.path.dirname(PKG)), "n_steps": model.n_steps,
           "n_params": model.n_params, "psnr_db": info["psnr_db"], "ms": info["ms"], "fallback": info["fallback"],
           "residual_learned": info["residual_learned"],
           "residual_plain_same_pairs": info["residual_plain_same_pairs"],
           "db_vs_tvbr_final": info["psnr_db"] - curve["final_psnr_db"],
           "tvbr_db_at_learned_time": psnr_at_time({"_psnr": np.asarray(curve["psnr"], dtype=np.float64),
                                                    "_t_ms": np.asarray(curve["t_ms"], dtype=np.float64)}, info["ms"]),
           "speedup_vs_tvbr_target_time": curve["t_target_ms"] / info["ms"],
           "speedup_vs_tvbr_total": curve["total_ms"] / info["ms"],
           "within_0p5_db": bool(info["psnr_db"] >= curve["target_psnr_db"])}
    if log:
        log(f"learned ({model.n_steps} steps): {info['psnr_db']:.2f} dB in {info['ms']:.0f} ms "
            f"({out['db_vs_tvbr_final']:+.2f} dB vs TV+Br, {out['speedup_vs_tvbr_target_time']:.1f}x faster than its "
            f"time to target), fallback {info['fallback']}")
    if rows:
        dbs = [out["db_vs_tvbr_final"]] + [r["db_vs_tvbr"] for r in rows]
        sps = [out["speedup_vs_tvbr_target_time"]] + [r["speedup_vs_target_time"] for r in rows]
        out["held_out"] = [{k: r[k] for k in ("seed", "tvbr_final_db", "tvbr_t_target_ms", "learned_db", "learned_ms",
                                              "db_vs_tvbr", "speedup_vs_target_time", "tvbr_db_at_learned_time",
                                              "fallback")} for r in rows]
        out["phantoms"] = len(dbs)
        out["mean_db_vs_tvbr_final"] = float(np.mean(dbs))
        out["mean_speedup_vs_tvbr_target_time"] = float(np.mean(sps))
        out["fallbacks"] = int(info["fallback"]) + sum(int(r["fallback"]) for r in rows)
        out["mean_within_0p5_db"] = bool(out["mean_db_vs_tvbr_final"] >= -0.5)
        if log:
            log(f"learned over {len(dbs)} phantoms: " + ", ".join(f"{d:+.2f} dB / {v:.1f}x" for d, v in zip(dbs, sps))
                + f"; mean {out['mean_db_vs_tvbr_final']:+.2f} dB, {out['mean_speedup_vs_tvbr_target_time']:.1f}x")
    return out


def evaluate_only(path, n=128, sampling="hadamard", n_steps=8, seeds=(5004,), repeats=2, log=None):
    """The learned reconstruction of a saved model alone (no training, no TV+Br reference run): for
    each phantom seed, `repeats` runs of reconstruct_with_fallback with its concurrent plain-FISTA
    check (the first also loads code); returns per-seed PSNR, wall time of the last run, fallback
    and residuals."""
    from synthetic import gaussian_volume
    dev = torch.device("cuda:0")
    model = LearnedUNetRecon.load(path, dev)
    model = model.truncated(min(n_steps, model.n_steps))
    plan, ref_plan = make_plan(n, sampling), make_plan(n, sampling)
    x0 = torch.from_numpy(gaussian_volume(plan.vol_shape, 8).astype(np.float32)).to(dev)
    L = P.pat_power_iteration(plan, x0, 10)
    rows = []
    for seed in seeds:
        case = make_case(plan, seed, sampling)
        for _ in range(max(1, repeats)):
            _, info = reconstruct_with_fallback(model, plan, case["f"], L, case["lam_tv"], case["lam_br"],
                                                p_ref=case["p0"], ref_plan=ref_plan)
        rows.append({"seed": seed, "n_steps": model.n_steps, **info})
        if log:
            log(f"phantom {seed}: {info['psnr_db']:.2f} dB in {info['ms']:.0f} ms, fallback {info['fallback']}")
    ref_plan.close()
    plan.close()
    return rows


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="Train and evaluate the U-Net learned reconstruction.")
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--sampling", choices=["hadamard", "points"], default="hadamard")
    ap.add_argument("--train", type=int, default=24)
    ap.add_argument("--test", type=int, default=4)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=2)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--widths", default="16,32,64")
    ap.add_argument("--workers", type=int, default=2)
    ap.add_argument("--save", default=None, help="safetensors path ('default': the package's weights directory)")
    ap.add_argument("--eval-steps", default="", help="comma-separated step counts evaluated besides --steps")
    ap.add_argument("--init", default=None, help="safetensors model to continue training from")
    ap.add_argument("--train-seed0", type=int, default=1000, help="seed of the first training phantom")
    ap.add_argument("--evaluate", default=None,
                    help="evaluate this saved model ('default': the package's weights) on --seeds and exit")
    ap.add_argument("--seeds", default="5004", help="phantom seeds of --evaluate (comma-separated)")
    a = ap.parse_args(argv)
    widths = tuple(int(w) for w in a.widths.split(","))
    if a.evaluate:
        path = weights_path(a.n, a.sampling, widths) if a.evaluate == "default" else a.evaluate
        rows = evaluate_only(path, a.n, a.sampling, a.steps, tuple(int(x) for x in a.seeds.split(",") if x.strip()),
                             log=lambda m: print(m, file=sys.stderr, flush=True))
        print(json.dumps(rows), flush=True)
        return
    save = weights_path(a.n, a.sampling, widths) if a.save == "default" else a.save
    ev = [int(k) for k in a.eval_steps.split(",") if k.strip()]
    out = experiment(a.n, a.sampling, a.train, a.test, a.steps, widths, a.epochs, a.batch, a.lr, a.workers, save,
                     ev, log=lambda m: print(m, file=sys.stderr, flush=True), init=a.init, train_seed0=a.train_seed0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
