"""Workload for rocprofv3: the stencil network's fused inference alone.

A network with seeded random weights (scaled like its initialisation) maps
`--rows` seeded random feature rows, `--reps` times; the inputs are copied to
the device and the outputs back on each call (the kernel trace separates
them).  Prints the wall time per call.

    python3 -m paper_1804_02297_amd.profile_mlp --rows 8192 --reps 10
"""
from __future__ import annotations

import argparse
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rows", type=int, default=8192)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--seed", type=int, default=3)
    a = ap.parse_args()

    import numpy as np
    from paper_1804_02297_amd import binding
    from paper_1804_02297_amd.binding import Mlp

    binding.load()
    g = np.random.default_rng(a.seed)
    shapes = {"W1": (250, 256), "b1": (256,), "W2": (256, 256), "b2": (256,), "W3": (256, 468), "b3": (468,)}
    p = {k: (g.standard_normal(s) / np.sqrt(s[0]) if len(s) == 2 else 0.05 * g.standard_normal(s))
         for k, s in shapes.items()}
    net = Mlp(Mlp.flat(p))
    x = g.standard_normal((a.rows, 250)).astype(np.float32)
    for r in range(a.reps):
        t = time.perf_counter()
        y = net.forward(x)
        print(f"call {r}: {time.perf_counter() - t:.4f} s (host copies included), max |y| {np.abs(y).max():.3f}",
              flush=True)
    net.close()


if __name__ == "__main__":
    main()
