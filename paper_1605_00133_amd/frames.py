"""Independent problems at once: the frames of a dynamic (4D) scan, several
phantoms, or a sweep of lambda.

Each problem has its own plan and runs on its own stream (default priority), so
the GPU overlaps the time steps of different problems: a step of one problem
leaves phases where all of its blocks compute or all wait for memory, which the
blocks of another fill (two 128^3 problems run about 1.2x the operator rate of
one). pat_reconstruct synchronises its stream once per FISTA iteration, so each
reconstruction is driven by a host thread of its own; the library's calls
release the Python interpreter lock and keep no shared mutable state. All work
runs in the library; this module only orders streams and threads.
"""

import threading

import torch

from . import pat as P


def _streams(plans):
    cur = torch.cuda.current_stream(plans[0].device)
    streams = [torch.cuda.Stream(device=p.device) for p in plans]
    for s in streams:
        s.wait_stream(cur)   # inputs written on the caller's stream come first
    return cur, streams


def _join(cur, streams):
    for s in streams:
        cur.wait_stream(s)


def forward_all(plans, p0s, fs):
    """f_k = C A p0_k for every plan k, concurrently; ordered after and before the caller's stream."""
    cur, streams = _streams(plans)
    for plan, s, p0, f in zip(plans, streams, p0s, fs):
        with torch.cuda.stream(s):
            P.pat_forward(plan, p0, f)
    _join(cur, streams)


def adjoint_all(plans, fs, ps):
    """p_k = A^T C^T f_k for every plan k, concurrently."""
    cur, streams = _streams(plans)
    for plan, s, f, p in zip(plans, streams, fs, ps):
        with torch.cuda.stream(s):
            P.pat_adjoint(plan, f, p)
    _join(cur, streams)


def _warm(plans, fs, ps):
    """One short reconstruction per distinct plan shape on the calling thread, before
    any worker starts, so that the first launch of every kernel a reconstruction
    uses (and the runtime's loading of its code) happens on one thread and not
    concurrently in the workers. Writes only ps[k] of the first plan of each shape,
    which the workers overwrite."""
    seen = set()
    for plan, f, p in zip(plans, fs, ps):
        g = plan.grid
        key = (g.nx, g.ny, g.nz, g.nt, plan.kind)
        if key in seen:
            continue
        seen.add(key)
        P.pat_reconstruct(plan, f, p, 0.0, 1.0, n_outer=1, n_inner=1, n_prox=1, restart=False)


def reconstruct_all(plans, fs, ps, lams, Ls, workers=None, warm=True, **kwargs):
    """pat_reconstruct(plans[k], fs[k], ps[k], lams[k], Ls[k], **kwargs) for every k.
    `workers` host threads (default: one per problem), each with a stream of its
    own, take the problems in list order (put the largest first to balance mixed
    sizes). With more than one worker and `warm`, one short reconstruction per
    distinct plan shape runs first on the calling thread (_warm). Returns the
    list of logs. The first error raised by any problem is raised again here,
    after all workers have ended; problems not yet started by then are skipped."""
    n = len(plans)
    workers = n if workers is None else max(1, min(int(workers), n))
    if workers > 1 and warm:
        _warm(plans, fs, ps)
    cur, streams = _streams(plans[:workers])
    outs, errs = [None] * n, [None] * n
    lock = threading.Lock()
    nxt = [0]

    def work(w):
        with torch.cuda.stream(streams[w]):
            while True:
                with lock:
                    k = nxt[0]
                    if k >= n or any(e is not None for e in errs):
                        return
                    nxt[0] += 1
                try:
                    outs[k] = P.pat_reconstruct(plans[k], fs[k], ps[k], lams[k], Ls[k], **kwargs)
                except Exception as e:   # re-raised in the caller's thread
                    errs[k] = e

    threads = [threading.Thread(target=work, args=(w,)) for w in range(workers)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    _join(cur, streams)
    for e in errs:
        if e is not None:
            raise e
    return outs


# Largest graph captured here, in kernel nodes (estimated by graph_nodes). Graphs of up to
# about 60 000 nodes (two iterations of a 24-frame scan at 64^3-128^3) were built and replayed
# many times; building one of about 900 000 (thirty iterations of that scan in one graph)
# ended the process with a host segmentation fault whose cause in this code is not known, so
# larger graphs are refused and a long scan is captured as a sequence of graphs instead.
MAX_GRAPH_NODES = 1 << 16


def graph_nodes(nts, n_iter, n_prox):
    """Upper estimate of the kernel launches that n_iter TV+ FISTA iterations of frames with these
    Nt enqueue (line scheme): per iteration one forward and one adjoint application (Nt step
    launches each plus set-up), n_prox dual and primal prox launches, and a few vector kernels."""
    return sum(5 + int(n_iter) * (2 * int(nt) + 2 * int(n_prox) + 24) for nt in nts)


def max_iters_per_graph(nts, n_prox, budget=MAX_GRAPH_NODES):
    """The most iterations of all frames that one graph may hold (at least 1)."""
    per = graph_nodes(nts, 1, n_prox) - graph_nodes(nts, 0, n_prox)
    return max(1, (budget - graph_nodes(nts, 0, n_prox)) // per)


class CapturedScan:
    """Every frame's TV+ FISTA (n_iter iterations from 0, no restart) captured in HIP graphs
    (torch.cuda.CUDAGraph over pat_fista_enqueue_from): each graph holds `iters_per_graph`
    iterations of ALL frames, frame k on branch k % branches (the branches join at the
    graph's end); replay() launches the graphs in order on the current stream. With
    iters_per_graph = n_iter (the default) the whole scan is one graph; a graph of more than
    MAX_GRAPH_NODES estimated launches is refused. The parts continue each other exactly, so
    the result does not depend on the split. Plans must use the line scheme (the slab scheme
    refuses capture). Outputs ps[k] and the per-iteration logs [n_iter, 2] (sum r^2, TV) are
    overwritten by each replay; data are read from fs[k] at replay time."""

    def __init__(self, plans, fs, lams, Ls, n_iter, n_prox=50, branches=4, order=None, iters_per_graph=None):
        dev = plans[0].device
        self.plans, self.fs, self.n_iter = plans, fs, int(n_iter)
        self.order = list(range(len(plans))) if order is None else list(order)
        self.branches = max(1, min(int(branches), len(plans)))
        self.n_prox = int(n_prox)
        k_graph = max(1, self.n_iter) if iters_per_graph is None else int(iters_per_graph)
        if not 1 <= k_graph <= max(1, self.n_iter):
            raise ValueError(f"iters_per_graph must be in [1, {self.n_iter}]")
        nts = [pl.grid.nt for pl in plans]
        self.nodes_per_graph = graph_nodes(nts, k_graph, self.n_prox)
        if self.nodes_per_graph > MAX_GRAPH_NODES:
            raise ValueError(f"a graph of {k_graph} iterations of these frames would hold about "
                             f"{self.nodes_per_graph} kernel launches, more than the {MAX_GRAPH_NODES} supported; "
                             f"use iters_per_graph <= {max_iters_per_graph(nts, self.n_prox)}")
        self.parts = [(i0, min(k_graph, self.n_iter - i0)) for i0 in range(0, self.n_iter, k_graph)]
        self.ps = [torch.empty(pl.vol_shape, dtype=torch.float32, device=dev) for pl in plans]
        self.logs = [torch.zeros((self.n_iter, 2), dtype=torch.float64, device=dev) for _ in plans]
        self.args = [(float(lams[k]), float(Ls[k])) for k in range(len(plans))]
        side = [torch.cuda.Stream(device=dev) for _ in range(self.branches)]   # default priority

        def enqueue(i0, m):
            cur = torch.cuda.current_stream(dev)
            for s in side:
                s.wait_stream(cur)
            for j, k in enumerate(self.order):
                with torch.cuda.stream(side[j % self.branches]):
                    lam, L = self.args[k]
                    P.pat_fista_enqueue_from(self.plans[k], self.fs[k], self.ps[k], lam, L, i0, m, self.n_prox,
                                             "dirichlet", self.logs[k][i0:i0 + m])
            for s in side:
                cur.wait_stream(s)

        for i0, m in self.parts:            # eager run: first launches and code loading outside the capture
            enqueue(i0, m)
        torch.cuda.synchronize(dev)
        self.graphs = []
        for i0, m in self.parts:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                enqueue(i0, m)
            self.graphs.append(g)
        for pl in plans:
            pl.sync_stream()                # back to the caller's stream for eager use

    @property
    def graph(self):
        """The single graph of a scan captured in one part."""
        if len(self.graphs) != 1:
            raise AttributeError(f"this scan is captured in {len(self.graphs)} graphs")
        return self.graphs[0]

    def replay(self):
        for g in self.graphs:
            g.replay()

    def energies(self):
        """Per frame, the energy 1/2 ||C A x - f||^2 + lambda TV(x) after each iteration (host arrays)."""
        return [0.5 * lg[:, 0].cpu().numpy() + self.args[k][0] * lg[:, 1].cpu().numpy()
                for k, lg in enumerate(self.logs)]


def autotune_scan(plans, fs, lams, Ls, n_iter, n_prox=50, candidates=(1, 2, 4, 8), probe_iters=2, cache=None,
                  log=None):
    """Chooses the number of graph branches and the frame order (largest first, or sizes
    interleaved) of a CapturedScan by timing replays of graphs with `probe_iters`
    iterations; the choice is written to `cache` (a JSON path) if given. Returns
    (choice, timings)."""
    import json
    import time
    sizes = [pl.grid.nx for pl in plans]
    largest = sorted(range(len(plans)), key=lambda k: -sizes[k])
    inter = []
    buckets = {}
    for k in largest:
        buckets.setdefault(sizes[k], []).append(k)
    while any(buckets.values()):
        for n in sorted(buckets, reverse=True):
            if buckets[n]:
                inter.append(buckets[n].pop(0))
    timings = []
    for order_name, order in (("largest_first", largest), ("interleaved", inter)):
        for b in candidates:
            if b > len(plans):
                continue
            scan = CapturedScan(plans, fs, lams, Ls, probe_iters, n_prox, b, order)
            scan.replay()
            torch.cuda.synchronize()
            t = time.perf_counter()
            for _ in range(2):
                scan.replay()
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t) / 2
            timings.append({"order": order_name, "branches": b, "ms": ms})
            if log:
                log(f"autotune: {order_name}, {b} branches: {ms:.1f} ms per replay of {probe_iters} iterations")
            del scan
    best = min(timings, key=lambda r: r["ms"])
    choice = {"branches": best["branches"], "order": best["order"],
              "frame_order": largest if best["order"] == "largest_first" else inter,
              "sizes": sizes, "probe_iters": probe_iters, "n_iter": n_iter}
    if cache:
        with open(cache, "w") as fh:
            json.dump({"choice": choice, "timings": timings}, fh)
    return choice, timings


def _scan_setup(sizes, n_frames, rate, seed, lam_rel=None):
    """Frames of a moving vessel phantom (1 voxel per frame, 10 % amplitude pulsation), each
    on a grid drawn from `sizes` with its own random single-point mask keeping 1/rate of the
    plane, data C A p0 + 1 % noise, lambda = lam_rel sigma sqrt(Nt M_c) (default: the value
    for one 128^3 problem, 2e-3) and L by power iteration on the first frame of each size.
    Returns plans, phantoms, data, lambdas, Ls, {size: L}, the size of each frame (largest
    frames first)."""
    import numpy as np

    from synthetic import gaussian_data, gaussian_volume
    from synthetic import moving_vessel_frames

    lam_rel = 2e-3 if lam_rel is None else float(lam_rel)
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(seed)
    frame_n = [int(sizes[i]) for i in rng.integers(0, len(sizes), n_frames)]
    seqs = {n: moving_vessel_frames((n, n, n), 8, n_frames, 24 if n >= 64 else 6, 1.0, 4.0 if n >= 64 else 2.0, seed)
            for n in sorted(set(frame_n))}
    order = sorted(range(n_frames), key=lambda t: -frame_n[t])   # largest frames first
    plans, p0s, fs, lams, Ls = [], [], [], [], []
    L_of = {}
    for t in order:
        n = frame_n[t]
        nt = int(round(740 * n / 128))
        mc = n * n // rate
        idx = P.pat_make_rsp_mask(n * n, mc, 1000 + t)
        plan = P.Plan(P.make_grid(n, n, n, 100e-6, 1500.0, 20e-9, nt, 8), "points", mc, idx)
        p0 = torch.from_numpy(seqs[n][t].astype(np.float32)).to(dev)
        f = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
        P.pat_forward(plan, p0, f)
        sigma = 0.01 * float(f.abs().max())
        f += sigma * torch.from_numpy(gaussian_data(plan.data_shape, 2000 + t).astype(np.float32)).to(dev)
        if n not in L_of:
            x0 = torch.from_numpy(gaussian_volume(plan.vol_shape, 8).astype(np.float32)).to(dev)
            L_of[n] = P.pat_power_iteration(plan, x0, 10)
        plans.append(plan)
        p0s.append(p0)
        fs.append(f)
        lams.append(lam_rel * sigma * np.sqrt(nt * mc))
        Ls.append(L_of[n])
    return plans, p0s, fs, lams, Ls, L_of, [frame_n[t] for t in order]


def captured_dynamic_scan(sizes=(64, 96, 128), n_frames=24, iters=30, rate=8, n_prox=50, seed=1, tune=True,
                          cache=None, log=print):
    """The dynamic (4D) scan in HIP graphs: all frames' TV+ FISTA (`iters` iterations, no
    restart) captured once (CapturedScan, branches and order from autotune_scan), as many
    iterations of all frames per graph as MAX_GRAPH_NODES allows, and launched by one
    replay; against the same iterations run eagerly frame after frame (pat_reconstruct,
    restart off: equal bit for bit). Returns rates and PSNRs."""
    import time

    import numpy as np

    plans, p0s, fs, lams, Ls, L_of, frame_n = _scan_setup(sizes, n_frames, rate, seed)
    torch.cuda.synchronize()
    log(f"{n_frames} frames, sizes {dict((n, frame_n.count(n)) for n in sorted(set(frame_n)))}, L {L_of}")
    if tune:
        choice, timings = autotune_scan(plans, fs, lams, Ls, iters, n_prox, cache=cache, log=log)
    else:
        choice, timings = {"branches": 4, "frame_order": list(range(n_frames)), "order": "largest_first"}, []
    k_graph = min(iters, max_iters_per_graph([pl.grid.nt for pl in plans], n_prox))
    scan = CapturedScan(plans, fs, lams, Ls, iters, n_prox, choice["branches"], choice["frame_order"],
                        iters_per_graph=k_graph)
    scan.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    scan.replay()
    torch.cuda.synchronize()
    t_graph = time.perf_counter() - t0
    eager = [torch.empty(pl.vol_shape, dtype=torch.float32, device=f.device) for pl, f in zip(plans, fs)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pl, f, p, lam, L in zip(plans, fs, eager, lams, Ls):
        P.pat_reconstruct(pl, f, p, lam, L, n_outer=1, n_inner=iters, n_prox=n_prox, bc="dirichlet", restart=False)
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0
    same = all(torch.equal(a, b) for a, b in zip(scan.ps, eager))
    psnr = [P.pat_psnr(pl, p, p0) for pl, p, p0 in zip(plans, scan.ps, p0s)]
    log(f"graph: {t_graph:.2f} s ({n_frames / t_graph:.3f} frames/s), eager one after another: {t_eager:.2f} s "
        f"({n_frames / t_eager:.3f} frames/s), identical {same}")
    out = {"frames": n_frames, "sizes": sorted(set(frame_n)), "frame_sizes": frame_n, "iters": iters,
           "n_prox": n_prox, "graph_s": t_graph, "frames_per_s_graph": n_frames / t_graph, "eager_s": t_eager,
           "frames_per_s_eager": n_frames / t_eager, "speedup": t_eager / t_graph, "identical_to_eager": same,
           "graphs": len(scan.graphs), "iters_per_graph": k_graph, "graph_nodes_estimate": scan.nodes_per_graph,
           "autotune": {k: v for k, v in choice.items() if k != "frame_order"}, "autotune_timings": timings,
           "psnr_db_mean": float(np.mean(psnr)), "psnr_db_min": float(np.min(psnr))}
    del scan
    for pl in plans:
        pl.close()
    return out


def dynamic_scan(sizes=(64,), n_frames=24, iters=30, workers=4, rate=8, n_prox=50, seed=1, log=print):
    """A dynamic (4D) scan: n_frames frames of a moving vessel phantom, each on a
    grid drawn from `sizes` (dx = 100 um, c0 = 1500 m/s, CFL 0.3, Nt = 740 N / 128,
    8-cell PML), with an independent random single-point mask keeping 1/rate of the
    sensor pixels, data C A p0 + 1 % Gaussian noise, and `iters` TV+ FISTA
    iterations per frame (lambda as for one 128^3 problem, L by power iteration on
    the first frame of each size). The frames are reconstructed once one after
    another on one stream and once by `workers` concurrent workers; returns a dict
    with both rates (frames/s) and the per-frame PSNR against the true frame."""
    import time

    import numpy as np

    dev = torch.device("cuda:0")
    plans, p0s, fs, lams, Ls, L_of, frame_n = _scan_setup(sizes, n_frames, rate, seed)
    torch.cuda.synchronize()
    log(f"{n_frames} frames, sizes {dict((n, frame_n.count(n)) for n in sorted(set(frame_n)))}, L {L_of}")
    kw = dict(n_outer=1, n_inner=iters, n_prox=n_prox, bc="dirichlet", restart=True)
    _warm(plans, fs, [torch.empty(pl.vol_shape, dtype=torch.float32, device=dev) for pl in plans])
    res = {}
    for w in (1, workers):
        ps = [torch.empty(pl.vol_shape, dtype=torch.float32, device=dev) for pl in plans]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reconstruct_all(plans, fs, ps, lams, Ls, workers=w, warm=False, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[w] = (n_frames / dt, ps)
        log(f"workers {w}: {dt:.2f} s, {n_frames / dt:.3f} frames/s")
    psnr = [P.pat_psnr(pl, p, p0) for pl, p, p0 in zip(plans, res[workers][1], p0s)]
    same = all(torch.equal(a, b) for a, b in zip(res[1][1], res[workers][1]))
    for pl in plans:
        pl.close()
    return {"frames": n_frames, "sizes": sorted(set(frame_n)), "iters": iters, "workers": workers,
            "frames_per_s_one_stream": res[1][0], "frames_per_s": res[workers][0],
            "speedup": res[workers][0] / res[1][0], "identical": same,
            "psnr_db_mean": float(np.mean(psnr)), "psnr_db_min": float(np.min(psnr))}


def main(argv=None):
    import argparse
    import json
    import sys
    ap = argparse.ArgumentParser(description="Reconstruct the frames of a synthetic dynamic (4D) scan.")
    ap.add_argument("--sizes", default="64", help="comma-separated grid sizes drawn per frame (16, 32, 64, 96, 128)")
    ap.add_argument("--frames", type=int, default=24)
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--n-prox", type=int, default=50)
    ap.add_argument("--captured", action="store_true",
                    help="all frames as one captured HIP graph (autotuned branches and order)")
    ap.add_argument("--cache", default=None, help="JSON file receiving the autotuner's choice")
    a = ap.parse_args(argv)
    sizes = tuple(int(s) for s in a.sizes.split(","))
    lg = lambda m: print(m, file=sys.stderr, flush=True)
    if a.captured:
        out = captured_dynamic_scan(sizes, a.frames, a.iters, n_prox=a.n_prox, cache=a.cache, log=lg)
    else:
        out = dynamic_scan(sizes, a.frames, a.iters, a.workers, n_prox=a.n_prox, log=lg)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
