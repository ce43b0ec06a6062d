"""One forward + adjoint pair at 128^3 (the benchmark's operator workload), for profilers.

Run under rocprofv3 to attribute time and hardware counters to the propagator
kernels, e.g.
    rocprofv3 --kernel-trace --stats -d OUT -o pair -- python3 -m paper_1605_00133_amd.profile_pair
    rocprofv3 --pmc FETCH_SIZE -d OUT -o fetch -- python3 -m paper_1605_00133_amd.profile_pair
A copy kernel of known size (torch's device-to-device copy of 256 MiB) runs
first, so counter readings can be scaled by what the same counter reports
for a known number of bytes. --concurrent K runs K independent problems (own
plan, phantom and stream each) at once, so that the working set (about
0.5 GB per 128^3 problem) is well above the 256 MB last-level cache.
"""

import argparse
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--nt", type=int, default=740)
    ap.add_argument("--pairs", type=int, default=1)
    ap.add_argument("--fft-precision", type=int, choices=[32, 64], default=64)
    ap.add_argument("--sampling", choices=["points", "hadamard"], default="points")
    ap.add_argument("--scheme", choices=["line", "slab"], default="line")
    ap.add_argument("--concurrent", type=int, default=1)
    args = ap.parse_args()
    import torch
    from paper_1605_00133_amd import pat as P
    from synthetic import vessel_phantom
    dev = torch.device("cuda:0")
    # reference copy of a known size: 256 MiB read + 256 MiB written
    a = torch.empty(64 * 2**20, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    n, nt = args.n, args.nt
    npix, mc = n * n, (n * n) // 8
    if args.sampling == "points":
        idx, perm = P.pat_make_rsp_mask(npix, mc, 2), None
    else:
        perm, idx = P.pat_make_shd_pattern(npix, mc, 4)
    K = max(1, args.concurrent)
    plans, p0s, fs, ps = [], [], [], []
    for k in range(K):
        plan = P.Plan(P.make_grid(n, n, n, 100e-6, 1500.0, 20e-9, nt, 8), args.sampling, mc, idx, perm)
        plan.set_fft_precision(args.fft_precision)
        if args.fft_precision == 64:
            plan.set_scheme(args.scheme)
        plans.append(plan)
        p0s.append(torch.from_numpy(vessel_phantom((n, n, n), 8, 24, 1.0, 4.0, 1 + k).astype(np.float32)).to(dev))
        fs.append(torch.empty(plan.data_shape, dtype=torch.float32, device=dev))
        ps.append(torch.empty(plan.vol_shape, dtype=torch.float32, device=dev))
    streams = [torch.cuda.Stream(device=dev) for _ in range(K)]   # default priority
    torch.cuda.synchronize()
    for _ in range(args.pairs):
        for k in range(K):
            with torch.cuda.stream(streams[k]):
                P.pat_forward(plans[k], p0s[k], fs[k])
                P.pat_adjoint(plans[k], fs[k], ps[k])
    torch.cuda.synchronize()
    print(f"profile_pair: {args.pairs} pair(s) x {K} problem(s) at {n}^3 nt={nt} fft f{args.fft_precision} "
          f"{args.scheme} done", flush=True)


if __name__ == "__main__":
    main()
