"""One forward + adjoint pair at 128^3 (the benchmark's operator workload), for profilers.

Run under rocprofv3 to attribute time and hardware counters to the propagator
kernels, e.g.
    rocprofv3 --kernel-trace --stats -d OUT -o pair -- python3 -m paper_1605_00133_amd.profile_pair
    rocprofv3 --pmc FETCH_SIZE -d OUT -o fetch -- python3 -m paper_1605_00133_amd.profile_pair
A copy kernel of known size (torch's device-to-device copy of 256 MiB) runs
first, so counter readings can be scaled by what the same counter reports
for a known number of bytes.
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
    plan = P.Plan(P.make_grid(n, n, n, 100e-6, 1500.0, 20e-9, nt, 8), args.sampling, mc, idx, perm)
    plan.set_fft_precision(args.fft_precision)
    if args.fft_precision == 64:
        plan.set_scheme(args.scheme)
    p0 = torch.from_numpy(vessel_phantom((n, n, n), 8, 24, 1.0, 4.0, 1).astype(np.float32)).to(dev)
    f = torch.empty(plan.data_shape, dtype=torch.float32, device=dev)
    p = torch.empty(plan.vol_shape, dtype=torch.float32, device=dev)
    for _ in range(args.pairs):
        P.pat_forward(plan, p0, f)
        P.pat_adjoint(plan, f, p)
    torch.cuda.synchronize()
    print(f"profile_pair: {args.pairs} pair(s) at {n}^3 nt={nt} fft f{args.fft_precision} {args.scheme} done",
          flush=True)


if __name__ == "__main__":
    main()
