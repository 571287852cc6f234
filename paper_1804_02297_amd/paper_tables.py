"""The paper's table columns (Section 4: the three 2-D tables and Tables 4-6
in 3-D) measured on the GPU.

For each grid n (six points per wavelength, k = 2 pi (n + 1) / 6) and each
analogue of the paper's media (a Gaussian lens, a cube obstacle with a smooth
boundary, a randomly perturbed cube; ``inputs.PAPER_MEDIA``) with the paper's
incident field E^i = (0, 0, e^{i k x_1}), it runs the paper's method: the 27
class stencils, the sparse LU of S (complex128, on the GPU), and GMRES
restarted every 20 steps to a relative residual of 1e-6 with the FP64 apply.
Columns as in the paper: T_setup (stencil fit + factorisation, s), T_apply
(one application of the preconditioner, s), N_iter, T_solve (s).  The
paper's own rows (MATLAB, other hardware) are printed beside them from the
fixture of its tables.  Inputs are the seeded generators'; no oracle.

With ``--dim 2`` the same for the 2-D variant: the analogues of the paper's
2-D media (``inputs.PAPER_MEDIA_2D``), E^i = (0, e^{i k x_1}), the 9 class
stencils and the nested-dissection factor of S (complex128) in HBM, or on
host cores with ``--factor host``.

    python3 -m paper_1804_02297_amd.paper_tables --n 29 59
    python3 -m paper_1804_02297_amd.paper_tables --dim 2 --n 119 239 479 959
"""
from __future__ import annotations

import argparse
import json
import os
import time


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[29, 59])
    ap.add_argument("--dim", type=int, choices=(2, 3), default=3)
    ap.add_argument("--factor", choices=("gpu", "host"), default="gpu",
                    help="2-D: factor S in HBM (default) or on host cores")
    ap.add_argument("--restart", type=int, default=20)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--factor-prec", choices=("c128", "c64"), default="c128")
    a = ap.parse_args()

    import torch
    from paper_1804_02297_amd import binding
    from paper_1804_02297_amd import inputs as I

    binding.load()
    dev = torch.device("cuda:0")
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    with open(os.path.join(here, "tests", "golden", f"paper_tables_{a.dim}d.json")) as f:
        gold = json.load(f)["rows"]

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    rows = []
    if a.dim == 2:
        rows = run_2d(a, binding, I, dev, gold, timed)
    for n in (a.n if a.dim == 3 else []):
        k = I.paper_wavenumber(n)
        for name, gen in I.PAPER_MEDIA.items():
            m = torch.from_numpy(gen(n)).to(dev)
            plan = binding.Plan(n, k, m, max_rhs=1)
            g = plan.rhs_from_incident(torch.from_numpy(I.paper_incident(n, k)).to(dev))
            t_fit, _ = timed(lambda: plan.stencil_fit(0))
            t_fac, _ = timed(lambda: plan.factor_gpu(a.factor_prec))
            v = torch.randn_like(g)
            z = torch.empty_like(g)
            plan.precond(v, z)                                   # warm-up
            reps = 5
            t_app, _ = timed(lambda: [plan.precond(v, z) for _ in range(reps)])
            plan.solve(g, tol=a.tol, restart=a.restart)           # warm-up (workspaces)
            t_sol, (x, info, st) = timed(lambda: plan.solve(g, tol=a.tol, restart=a.restart))
            paper = [r for r in gold if r["medium"] == name and abs(r["k_over_2pi"] - k / (2 * 3.141592653589793)) < 1e-6]
            row = {"medium": name, "n": n, "k_over_2pi": round(k / (2 * 3.141592653589793), 3),
                   "N": 3 * n ** 3, "T_setup": round(t_fit + t_fac, 4), "T_apply": round(t_app / reps, 5),
                   "N_iter": info[0]["iters"], "T_solve": round(t_sol, 4), "rel_resid": info[0]["rel_resid"],
                   "status": st, "paper": paper[0] if paper else None}
            print(json.dumps(row), flush=True)
            rows.append(row)
            plan.close()
    print("| medium | k/2pi | N | T_setup | T_apply | N_iter | T_solve | paper N_iter | paper T_setup / T_apply / T_solve |")
    print("|---|---|---|---|---|---|---|---|---|")
    for r in rows:
        p = r["paper"] or {}
        size = f"3x{r['n']}^3" if a.dim == 3 else f"2x{r['n']}^2"
        print(f"| {r['medium']} | {r['k_over_2pi']:g} | {size} | {r['T_setup']:.3f} | {r['T_apply']:.4f} | "
              f"{r['N_iter']} | {r['T_solve']:.3f} | {p.get('N_iter', '-')} | "
              f"{p.get('T_setup', '-')} / {p.get('T_apply', '-')} / {p.get('T_solve', '-')} |")


def run_2d(a, binding, I, dev, gold, timed):
    import math
    import torch
    rows = []
    for n in a.n:
        k = I.paper_wavenumber(n)
        for name, gen in I.PAPER_MEDIA_2D.items():
            m = torch.from_numpy(gen(n)).to(dev)
            plan = binding.Plan2(n, k, m, max_rhs=1)
            g = plan.rhs_from_incident(torch.from_numpy(I.paper_incident2(n, k)).to(dev))
            t_fit, _ = timed(plan.stencil_fit)
            if a.factor == "gpu":
                t_fac, _ = timed(lambda: plan.factor_gpu(a.factor_prec))
            else:
                t_fac, _ = timed(lambda: plan.factor(a.factor_prec))
            v = torch.randn_like(g)
            z = torch.empty_like(g)
            plan.precond(v, z)
            reps = 5
            t_app, _ = timed(lambda: [plan.precond(v, z) for _ in range(reps)])
            plan.solve(g, tol=a.tol, restart=a.restart)
            t_sol, (x, info, st) = timed(lambda: plan.solve(g, tol=a.tol, restart=a.restart))
            kk = k / (2 * math.pi)
            paper = [r for r in gold if r["medium"] == name and abs(r["k_over_2pi"] - kk) < 1e-6]
            row = {"medium": name, "n": n, "k_over_2pi": round(kk, 3), "N": 2 * n * n,
                   "T_setup": round(t_fit + t_fac, 4), "T_fit": round(t_fit, 4), "T_factor": round(t_fac, 4),
                   "T_apply": round(t_app / reps, 5), "N_iter": info[0]["iters"], "T_solve": round(t_sol, 4),
                   "rel_resid": info[0]["rel_resid"], "status": st, "paper": paper[0] if paper else None}
            print(json.dumps(row), flush=True)
            rows.append(row)
            plan.close()
    return rows


if __name__ == "__main__":
    main()
