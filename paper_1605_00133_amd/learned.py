"""A learned update step on top of the paper's gradient (not part of its method).

K unrolled steps, each with a network of its own:
    z_k     = p_k - eta A^T C^T (C A p_k - f)        gradient step, eta = 1.8 / L (eq. BP, App. B)
    p_{k+1} = max(0, z_k + net_k([p_k, z_k]))        learned correction, positivity kept
from p_0 = 0. net_k is conv(2->c, ReLU) -> conv(c->c, ReLU) -> conv(c->1), 3x3x3
convolutions with BF16 matrix-core products (paper_1605_00133_amd.nn). The nets
are trained one step after another (greedy): net_k maps the training set's z_k
to the targets, the plain TV(+Bregman) reconstructions of the same data, in mean
squared error; the next step then starts from the trained step's output.

The operator, the convolutions and their gradients, Adam and, in the learned
iteration itself (reconstruct, CapturedReconstruct), every elementwise step
(residual, gradient step, the input stacking, the correction and its clamp:
pat_axpby) run in libpat's kernels. Training differentiates the step with torch
autograd (the convolutions' backward is libpat's); there the same elementwise
steps and the squared-error loss are torch operations, with the same FP32
arithmetic as pat_axpby.
"""

import math

import torch

from . import nn
from . import pat as P


def _he(shape, gen, gain=1.0):
    fan_in = shape[1] * 27
    return (torch.randn(shape, generator=gen) * (gain * math.sqrt(2.0 / fan_in))).float()


class LearnedUpdate:
    """Weights of K unrolled steps (device tensors)."""

    def __init__(self, n_steps=5, channels=16, seed=0, device="cuda:0"):
        g = torch.Generator().manual_seed(seed)
        c = channels
        self.params = []
        for _ in range(n_steps):
            step = [_he((c, 2, 3, 3, 3), g), torch.zeros(c), _he((c, c, 3, 3, 3), g), torch.zeros(c),
                    _he((1, c, 3, 3, 3), g, 0.1), torch.zeros(1)]
            self.params.append([t.to(device).contiguous() for t in step])

    @property
    def n_steps(self):
        return len(self.params)

    def net(self, k, inp):
        w1, b1, w2, b2, w3, b3 = self.params[k]
        h = nn.conv3d(inp, w1, b1, relu=True)
        h = nn.conv3d(h, w2, b2, relu=True)
        return nn.conv3d(h, w3, b3)

    def step(self, k, p, z):
        """p_{k+1} from [B, 1, nz, ny, nx] iterates p and gradient steps z. Under autograd (training)
        the elementwise glue is torch's; otherwise pat_axpby (the same FP32 operations)."""
        if torch.is_grad_enabled() and any(t.requires_grad for t in self.params[k]):
            return torch.clamp_min(z + self.net(k, torch.cat([p, z], dim=1).contiguous()), 0.0)
        x = torch.empty((p.shape[0], 2) + tuple(p.shape[2:]), dtype=torch.float32, device=p.device)
        for b in range(p.shape[0]):
            nn.axpby(p[b, 0].contiguous(), None, 1.0, out=x[b, 0])
            nn.axpby(z[b, 0].contiguous(), None, 1.0, out=x[b, 1])
        return nn.axpby(z.contiguous(), self.net(k, x), 1.0, 1.0, clamp0=True)


def gradient_step(plan, f, p, eta):
    """z = p - eta A^T C^T (C A p - f) for one volume [nz, ny, nx] (library operator and pat_axpby)."""
    r = torch.empty(plan.data_shape, dtype=torch.float32, device=p.device)
    P.pat_forward(plan, p.contiguous(), r)
    nn.axpby(r, f, 1.0, -1.0, out=r)
    g = torch.empty(plan.vol_shape, dtype=torch.float32, device=p.device)
    P.pat_adjoint(plan, r, g)
    return nn.axpby(p.contiguous(), g, 1.0, -eta)


def reconstruct(model, plan, f, L):
    """p_K of the unrolled learned iteration for data f [nt, mc]; K operator pairs."""
    eta = 1.8 / L
    p = torch.zeros(plan.vol_shape, dtype=torch.float32, device=f.device)
    with torch.no_grad():
        for k in range(model.n_steps):
            z = gradient_step(plan, f, p, eta)
            p = model.step(k, p[None, None], z[None, None])[0, 0].contiguous()
    return p


class CapturedReconstruct:
    """The K unrolled steps captured once as a HIP graph (torch.cuda.CUDAGraph):
    every operator pair, convolution and elementwise step of reconstruct() for
    data placed in self.f, replayed with one launch. The graph holds kernel
    launches only (no memory set or copy nodes). The plan must not be used by
    other work while a replay runs."""

    def __init__(self, model, plan, L, device="cuda:0"):
        self.plan = plan
        self.f = torch.zeros(plan.data_shape, dtype=torch.float32, device=device)
        s = torch.cuda.Stream(device=device)
        s.wait_stream(torch.cuda.current_stream(device))
        with torch.cuda.stream(s):            # warm-up outside the capture (allocations, code loading)
            reconstruct(model, plan, self.f, L)
        torch.cuda.current_stream(device).wait_stream(s)
        torch.cuda.synchronize(device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.p = reconstruct(model, plan, self.f, L)
        plan.sync_stream()                    # back to the caller's stream for eager use

    def __call__(self, f):
        """p_K for data f [nt, mc]; returns the graph's output tensor (overwritten by the next call)."""
        self.f.copy_(f)
        self.graph.replay()
        return self.p


def train(model, plan, fs, targets, L, epochs=150, batch=8, lr=2e-3, log=None):
    """Greedy training on data fs[i] and targets[i] (lists of device tensors);
    returns the final mean squared error of each step."""
    eta = 1.8 / L
    n = len(fs)
    ps = [torch.zeros(plan.vol_shape, dtype=torch.float32, device=fs[0].device) for _ in range(n)]
    T = torch.stack(targets)[:, None].contiguous()
    losses = []
    gen = torch.Generator().manual_seed(1)
    for k in range(model.n_steps):
        with torch.no_grad():
            Z = torch.stack([gradient_step(plan, f, p, eta) for f, p in zip(fs, ps)])[:, None].contiguous()
            Pk = torch.stack(ps)[:, None].contiguous()
        params = model.params[k]
        m = [torch.zeros_like(t) for t in params]
        v = [torch.zeros_like(t) for t in params]
        t_adam = 0
        for ep in range(epochs):
            perm = torch.randperm(n, generator=gen)
            for s in range(0, n, batch):
                idx = perm[s:s + batch].to(Z.device)
                for t in params:
                    t.requires_grad_(True)
                    t.grad = None
                out = model.step(k, Pk[idx], Z[idx])
                loss = ((out - T[idx]) ** 2).mean()
                loss.backward()
                t_adam += 1
                with torch.no_grad():
                    for t, mt, vt in zip(params, m, v):
                        nn.adam_step_(t.data, t.grad.contiguous(), mt, vt, t_adam, lr=lr)
                for t in params:
                    t.requires_grad_(False)
                    t.grad = None
        with torch.no_grad():
            out = torch.cat([model.step(k, Pk[s:s + batch], Z[s:s + batch]) for s in range(0, n, batch)])
            mse = float(((out - T) ** 2).mean())
            ps = [o[0].contiguous() for o in out]
        losses.append(mse)
        if log:
            log(f"step {k}: training MSE {mse:.3e}")
    return losses


def experiment(n=32, n_train=24, n_test=6, n_steps=5, epochs=150, channels=16, workers=4, seed=1, log=None):
    """Trains and evaluates the learned update on synthetic data: vessel phantoms on
    an n^3 grid (8-cell PML, dx = 100 um, c0 = 1500 m/s, CFL 0.3, Nt = 740 n / 128),
    one random single-point mask keeping a quarter of the sensor pixels, data
    C A p0 + 1 % Gaussian noise. Targets: TV+Br (lambda = 10 lambda0, 5 x 50 FISTA
    iterations, lambda0 = 2e-3 sigma sqrt(Nt M_c)). On the held-out phantoms it
    reports the PSNR (eq. PSNR) and wall time of the learned iteration (n_steps
    operator pairs), of plain TV+ FISTA with the same number of pairs, and of the
    TV+Br targets."""
    import time

    import numpy as np

    from synthetic import gaussian_data, gaussian_volume, vessel_phantom

    from .frames import reconstruct_all

    dev = torch.device("cuda:0")
    nt, mc = int(round(740 * n / 128)), n * n // 4
    idx = P.pat_make_rsp_mask(n * n, mc, 7)
    grid = P.make_grid(n, n, n, 100e-6, 1500.0, 20e-9, nt, 8)
    total = n_train + n_test
    plans = [P.Plan(grid, "points", mc, idx) for _ in range(total)]
    nv, rmax = (6, 2.0) if n <= 32 else (24, 4.0)
    p0s, fs, lams = [], [], []
    for i in range(total):
        p0 = torch.from_numpy(vessel_phantom((n, n, n), 8, nv, 1.0, rmax, seed * 1000 + i).astype(np.float32)).to(dev)
        f = torch.empty(plans[0].data_shape, dtype=torch.float32, device=dev)
        P.pat_forward(plans[0], p0, f)
        sigma = 0.01 * float(f.abs().max())
        f += sigma * torch.from_numpy(gaussian_data(f.shape, seed * 1000 + 500 + i).astype(np.float32)).to(dev)
        p0s.append(p0)
        fs.append(f)
        lams.append(2e-3 * sigma * math.sqrt(nt * mc))
    x0 = torch.from_numpy(gaussian_volume(plans[0].vol_shape, 8).astype(np.float32)).to(dev)
    L = P.pat_power_iteration(plans[0], x0, 20)
    targets = [torch.empty(plans[0].vol_shape, dtype=torch.float32, device=dev) for _ in range(total)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for c0 in range(0, total, workers):   # in chunks, so that progress is reported on large grids
        c1 = min(c0 + workers, total)
        reconstruct_all(plans[c0:c1], fs[c0:c1], targets[c0:c1], [10 * lam for lam in lams[c0:c1]], [L] * (c1 - c0),
                        workers=workers, n_outer=5, n_inner=50, n_prox=50)
        if log and total > workers:
            log(f"targets {c1}/{total}")
    torch.cuda.synchronize()
    if log:
        log(f"{total} TV+Br targets in {time.perf_counter() - t0:.1f} s, L = {L:.4e}")
    model = LearnedUpdate(n_steps, channels, seed, dev)
    t0 = time.perf_counter()
    losses = train(model, plans[0], fs[:n_train], targets[:n_train], L, epochs=epochs, log=log)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        return out, time.perf_counter() - t

    res = {"learned": [], "plain_same_pairs": [], "tv_bregman": [], "t_learned": 0.0, "t_learned_graph": 0.0,
           "t_plain": 0.0, "t_tvbr": 0.0, "graph_equals_eager": True}
    cap = CapturedReconstruct(model, plans[n_train], L, dev)
    for i in range(n_train, total):
        pl, p0, f = plans[i], p0s[i], fs[i]
        p, dt = timed(lambda: reconstruct(model, pl, f, L))
        res["learned"].append(P.pat_psnr(pl, p, p0))
        res["t_learned"] += dt
        pg, dt = timed(lambda: cap(f))
        res["t_learned_graph"] += dt
        res["graph_equals_eager"] = res["graph_equals_eager"] and bool(torch.equal(pg, p))
        q = torch.empty(pl.vol_shape, dtype=torch.float32, device=dev)
        _, dt = timed(lambda: P.pat_reconstruct(pl, f, q, lams[i], L, n_outer=1, n_inner=n_steps, n_prox=50))
        res["plain_same_pairs"].append(P.pat_psnr(pl, q, p0))
        res["t_plain"] += dt
        _, dt = timed(lambda: P.pat_reconstruct(pl, f, q, 10 * lams[i], L, n_outer=5, n_inner=50, n_prox=50))
        res["tv_bregman"].append(P.pat_psnr(pl, q, p0))
        res["t_tvbr"] += dt
    for pl in plans:
        pl.close()
    out = {k: (float(np.mean(v)) if isinstance(v, list) else v) for k, v in res.items()}
    del cap
    out.update({"n": n, "n_train": n_train, "n_test": n_test, "n_steps": n_steps, "epochs": epochs,
                "train_s": train_s, "train_mse": losses, "speedup_vs_tvbr": res["t_tvbr"] / res["t_learned"],
                "speedup_vs_tvbr_graph": res["t_tvbr"] / res["t_learned_graph"],
                "psnr_db_learned_minus_tvbr": float(np.mean(res["learned"]) - np.mean(res["tv_bregman"])),
                "psnr_db_learned_minus_plain": float(np.mean(res["learned"]) - np.mean(res["plain_same_pairs"]))})
    return out


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="Train and evaluate the learned update step on synthetic data.")
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--train", type=int, default=24)
    ap.add_argument("--test", type=int, default=6)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--channels", type=int, default=16)
    a = ap.parse_args(argv)
    out = experiment(a.n, a.train, a.test, a.steps, a.epochs, a.channels,
                     log=lambda m: print(m, file=sys.stderr, flush=True))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
