"""Driver for rocprofv3 runs of the Nystrom apply (kernel trace and HBM counters).

    python -m paper_1804_02297_amd.profile_apply --n 128 --nrhs 8 --prec c64 --reps 5
    python -m paper_1804_02297_amd.profile_apply --dim 2 --n 959 --nrhs 8 --prec c64 --reps 5

Runs `reps` applies of the benchmark workload (seeded sum-of-Gaussians
contrast, random fields; with --dim 2 the 2-D variant on the perturbed-square
analogue) and then `reps` plain device copies of a known size
(torch's copy kernel, 1 GiB) that calibrate the FETCH_SIZE / WRITE_SIZE
counters: a copy of S bytes must read S and write S.
"""
from __future__ import annotations

import argparse
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--prec", default="c64", choices=["c64", "c128", "mixed"])
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--dim", type=int, default=3, choices=(2, 3))
    ap.add_argument("--tune", action="store_true", help="use the autotuner's launch choice (as bench.py does)")
    ap.add_argument("--choice", default="", help="launch choice chunk,kmul_w,half_runs,persist (3-D)")
    args = ap.parse_args()
    import torch

    from paper_1804_02297_amd import binding
    from paper_1804_02297_amd import inputs as I
    binding.load()
    dev = torch.device("cuda:0")
    n, B = args.n, args.nrhs
    dt = torch.complex64 if args.prec == "c64" else torch.complex128
    g = torch.Generator(device=dev).manual_seed(7)
    if args.dim == 3:
        m = torch.from_numpy(I.medium_bumps(n, 3)).to(dev)
        plan = binding.Plan(n, I.wavenumber_for(n), m, max_rhs=B)
        x = torch.randn((B, 3, n, n, n), dtype=dt, device=dev, generator=g)
    else:
        m = torch.from_numpy(I.medium2_perturbed_square(n, 3)).to(dev)
        plan = binding.Plan2(n, I.paper_wavenumber(n), m, max_rhs=B)
        x = torch.randn((B, 2, n, n), dtype=dt, device=dev, generator=g)
    y = torch.empty_like(x)
    if args.tune and args.dim == 3:
        print("profile_apply tuned:", plan.tune(B, args.prec), flush=True)
    if args.choice and args.dim == 3:
        plan.set_tune(args.prec, *[int(v) for v in args.choice.split(",")])
    for _ in range(args.reps):
        plan.apply(x, y, prec=args.prec)
    torch.cuda.synchronize()
    nbytes = args.copy_mib << 20
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(args.reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"profile_apply done: dim={args.dim} n={n} nrhs={B} prec={args.prec} reps={args.reps} copy={nbytes} B", flush=True)
    plan.close()


if __name__ == "__main__":
    main()
