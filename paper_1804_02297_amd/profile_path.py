"""Workload for rocprofv3: the preconditioner path at one grid size.

Runs, once each and in this order: plan creation (Khat), the class fit, the
exact per-point fit, training samples from one other medium, network training,
the learned fit, the factorisation (host or GPU, complex128 or complex64) and
one block FGMRES solve (mixed precision, 2 polarisations x ndirs directions).
With --fit class only the class fit runs before the factorisation.  Prints
one line per step with its wall time.  Inputs are the seeded generators'; the
oracle is not used.

    python3 -m paper_1804_02297_amd.profile_path --n 32 --dirs 8 --train-steps 200
    python3 -m paper_1804_02297_amd.profile_path --n 64 --dirs 32 --fit class --factor gpu --factor-prec c64
"""
from __future__ import annotations

import argparse
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=32)
    ap.add_argument("--dirs", type=int, default=8)
    ap.add_argument("--train-steps", type=int, default=200)
    ap.add_argument("--fit", choices=("learned", "class"), default="learned")
    ap.add_argument("--factor", choices=("host", "gpu"), default="host")
    ap.add_argument("--factor-prec", choices=("c128", "c64"), default="c128")
    a = ap.parse_args()

    import numpy as np
    import torch
    from paper_1804_02297_amd import binding
    from paper_1804_02297_amd import inputs as I

    binding.load()
    dev = torch.device("cuda:0")
    n = a.n
    k = I.wavenumber_for(n)
    nb = 2 * a.dirs
    interior = [(p * n + q) * n + r for p in range(1, n - 1) for q in range(1, n - 1) for r in range(1, n - 1)]

    def step(name, fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        print(f"{name}: {time.perf_counter() - t0:.4f} s", flush=True)
        return out

    g = np.random.default_rng(7)
    params = np.concatenate([
        (g.standard_normal((250, 256)) * np.sqrt(2 / 250)).ravel(), np.zeros(256),
        (g.standard_normal((256, 256)) * np.sqrt(2 / 256)).ravel(), np.zeros(256),
        (g.standard_normal((256, 468)) * np.sqrt(2 / 256)).ravel(), np.zeros(468)]).astype(np.float32)
    net = binding.Mlp(params)
    if a.fit == "learned":
        pt = step("plan (training medium)",
                  lambda: binding.Plan(n, k, torch.from_numpy(I.medium_bumps(n, 1000)).to(dev)))
        step("training samples", lambda: net.add_samples(pt, interior))
        pt.close()
        step("training", lambda: net.train(a.train_steps, batch=1024, lr=1e-3, seed=0))
    plan = step("plan", lambda: binding.Plan(n, k, torch.from_numpy(I.medium_bumps(n, 3)).to(dev), max_rhs=nb))
    step("class fit", lambda: plan.stencil_fit(0))
    if a.fit == "learned":
        step("point fit", lambda: plan.stencil_fit(1))
        nfb = step("learned fit", lambda: plan.stencil_fit_learned(net))
        print(f"fallback points: {nfb} of {len(interior)}", flush=True)
    if a.factor == "gpu":
        step(f"GPU factor ({a.factor_prec})", lambda: plan.factor_gpu(a.factor_prec))
    else:
        step(f"host factor ({a.factor_prec})", lambda: plan.factor(a.factor_prec))
    dirs, pols = I.fibonacci_incident_set(a.dirs)
    Ei = torch.from_numpy(I.plane_waves(n, k, dirs, pols)).to(dev)
    gg = plan.rhs_from_incident(Ei)
    x, infos, st = step("block solve (mixed)", lambda: plan.solve(gg, tol=1e-8, prec="mixed"))
    print(f"status {st}, iterations {max(i['iters'] for i in infos)}, "
          f"max rel resid {max(i['rel_resid'] for i in infos):.2e}", flush=True)
    plan.close()
    net.close()


if __name__ == "__main__":
    main()
