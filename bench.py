#!/usr/bin/env python3
"""Benchmark: Munknowns/s of the Lippmann-Schwinger (Nystrom) apply at 128^3.

One step = one application y = x + K * (m x) (Eq. (5)) to a batch of 8
right-hand sides on the 128^3 grid (6.29M unknowns each; padded FFT 256^3),
with FP32 FFTs (complex64 fields), through the C ABI.  Inputs are seeded
synthetic fields and a sum-of-Gaussians contrast, resident in HBM before the
timed region starts.

Prints one JSON line with the throughput, a roofline entry for the dominant
kernel (algorithmic bytes per launch / average launch time, from HIP events
recorded between the passes on the stream the kernels run on), the FP64 and
mixed-precision rates, and the CPU oracle's apply timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X published HBM3E bandwidth
PASS_NAMES = ["dim1_fwd_mscale", "dim2_fwd", "dim3_fft_symbol_ifft", "dim2_inv", "dim1_inv_identity"]
KERNEL_NAMES = ["col_fft_kernel (mode 0)", "col_fft_kernel (mode 1)", "kmul_kernel",
                "col_fft_kernel (mode 2)", "col_fft_kernel (mode 3)"]


# HBM traffic of the dominant kernel (kmul_kernel, pass 3) per launch at n=128,
# 8 rhs, complex64, from rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by the 1 GiB
# copy calibration (read = 2.0 x FETCH_SIZE, write = 1.0 x WRITE_SIZE), valid
# only while the apply sources are the ones that were profiled.
MEASURED_TRAFFIC = {
    "sources": ["fft_kernels.h", "fft_apply.hip", "fft_inst_e.hip", "common.h", "cplx.h"],
    "sha256": "0a5f922aa79cf46908be21d9e0d170265055a3eede956f350db5b0f55b453bf4",
    "workload": (128, 8, "c64"),
    "bytes": 3.3265e9,
    "profile": "profiles/ls_apply_n128_b8_c64.md",
}

# HBM bytes of one 2-D column-pass launch (pass_b_kernel, n = 959, 8 rhs,
# complex64) from rocprofv3 FETCH_SIZE / WRITE_SIZE, calibrated as above;
# reported only while the sources are the measured ones.
MEASURED_TRAFFIC_2D = {
    "sources": ["twod.hip", "twod.h", "cplx.h"],
    "sha256": "cf6e2a189cd9b62519a9921a5757e0a3f4e7ffea85c18c279ef83f30936b6f2f",
    "workload": (959, 8, "c64"),
    "bytes": 9.343e8,
    "profile": "profiles/ls2_apply_n959_b8_c64.md",
}


def measured_traffic(n: int, B: int, prec: str, table=None):
    import hashlib
    table = table or MEASURED_TRAFFIC
    h = hashlib.sha256()
    for f in table["sources"]:
        with open(os.path.join(ROOT, "paper_1804_02297_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != table["sha256"] or (n, B, prec) != table["workload"]:
        return None
    return table["bytes"]


def pass_bytes(n: int, P: int, B: int, s: int, s_io: int) -> list[float]:
    """Algorithmic HBM bytes of each pass for B right-hand sides.

    s: bytes per complex in the FFT passes, s_io: bytes per complex of x and y.
    pass 1 reads x and m (once per component) and writes P n^2 per component;
    pass 3 also reads the octant symbol (6 (P/2+1)^3 values) once per launch.
    """
    n3 = n ** 3
    H = P // 2 + 1
    c = 3 * B
    return [
        c * (n3 * s_io + n3 * s + P * n * n * s),
        c * (P * n * n * s + P * P * n * s),
        c * (2 * P * P * n * s) + 6 * H ** 3 * s,
        c * (P * P * n * s + P * n * n * s),
        c * (P * n * n * s + 2 * n3 * s_io),
    ]


def host_cores() -> int:
    """Host threads available to this process (the machine's CPU share, at most 16)."""
    try:
        c = len(os.sched_getaffinity(0))
    except AttributeError:
        c = os.cpu_count() or 1
    return max(1, min(16, c))


def cpu_baseline(n: int, seconds: float = 8.0):
    """The oracle's FFT apply on the host, one rhs at a time, ~seconds of work,
    with one FFT worker (the headline value) and with every host core."""
    import numpy as np
    import scipy.fft
    from oracle import operator as op
    from paper_1804_02297_amd import inputs as I
    k = I.wavenumber_for(n)
    m = I.medium_bumps(n, 3)
    x = I.random_field(1, n, 5)
    t0 = time.perf_counter()
    Kh = op.kernel_symbol(n, k)
    t_setup = time.perf_counter() - t0

    def run(workers):
        reps, t_apply = 0, 0.0
        with scipy.fft.set_workers(workers):
            while t_apply < seconds and reps < 20:
                t0 = time.perf_counter()
                op.apply_fft(n, k, m, x, Kh)
                t_apply += time.perf_counter() - t0
                reps += 1
        return reps, t_apply / reps

    reps, per = run(1)
    cores = host_cores()
    reps_all, per_all = run(cores)
    return {"value": round(3 * n ** 3 / per / 1e6, 3), "unit": "Munknowns/s", "cores": 1,
            "kind": "oracle",
            "sample": f"oracle FFT apply (scipy.fft, 1 worker, FP64) of 1 rhs at n={n}, "
                      f"{reps} repetitions, {per:.2f} s each; symbol setup {t_setup:.1f} s untimed",
            "all_cores": {"value": round(3 * n ** 3 / per_all / 1e6, 3), "unit": "Munknowns/s",
                          "cores": cores, "kind": "oracle",
                          "sample": f"the same apply with scipy.fft workers={cores} (the 3x3 symbol "
                                    f"product stays on one thread), {reps_all} repetitions, "
                                    f"{per_all:.2f} s each"}}


def cpu_baseline_solve(n: int = 16):
    """Per-rhs time to a 1e-8 residual of the oracle's plain FP64 path on the host
    (the paper's class fit by thin SVD, SciPy's sparse LU of S, the oracle's
    FGMRES(30) with its FFT apply), on one seeded plane wave: the CPU
    counterpart of the per-rhs solve metric.  Set-up is timed apart."""
    from oracle import fgmres as ofg
    from oracle import operator as op
    from oracle import sparse as osp
    from oracle import stencil as ost
    from paper_1804_02297_amd import inputs as I
    k = I.wavenumber_for(n)
    m = I.medium_single_bump(n, 0) if n == 16 else I.medium_bumps(n, 1)
    d, p = I.random_direction_and_polarisation(0)
    Ei = I.plane_waves(n, k, [d], [p])
    t0 = time.perf_counter()
    Kh = op.kernel_symbol(n, k)
    g = op.rhs_from_incident(n, k, m, Ei, Kh)[0]
    al, be, _ = ost.fit_all_classes(n, k)
    _progress(f"oracle solve n={n}: class fit done at {time.perf_counter() - t0:.0f} s")
    S, Q = osp.assemble(n, m, al, be)
    _progress(f"oracle solve n={n}: assembly done at {time.perf_counter() - t0:.0f} s, sparse LU next")
    P = osp.Preconditioner(S, Q)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, info = ofg.fgmres(lambda v: op.apply_fft(n, k, m, v, Kh), g, P, tol=1e-8, restart=30)
    t_solve = time.perf_counter() - t0
    return {"value": round(t_solve, 3), "unit": "s per rhs", "cores": 1, "kind": "oracle",
            "n": n, "iters": info["iters"], "rel_resid": float(f"{info['rel_resid']:.3e}"),
            "setup_s": round(t_setup, 2),
            "sample": f"oracle plain FP64 solve at n={n} ({3 * n ** 3} unknowns), 1 plane wave: "
                      f"FGMRES(30) to 1e-8 with SciPy splu of S (one thread) and the FFT apply "
                      f"(1 worker); set-up (symbol, 27 class SVDs, assembly, splu) {t_setup:.1f} s untimed"}


def cpu_baseline_2d(n: int = 959, seconds: float = 5.0):
    """The oracle's 2-D FFT apply on the host, one rhs at a time (the 2-D
    variant's counterpart of ``cpu_baseline``)."""
    from oracle import two_d as o2
    from paper_1804_02297_amd import inputs as I
    k = I.paper_wavenumber(n)
    m = I.medium2_perturbed_square(n, 3)
    x = I.random_field2(1, n, 5)[0]
    t0 = time.perf_counter()
    sym = o2.symbol2(n, k)
    t_setup = time.perf_counter() - t0
    reps, t_apply = 0, 0.0
    while t_apply < seconds and reps < 20:
        t0 = time.perf_counter()
        o2.apply_fft2(n, k, m, x, sym)
        t_apply += time.perf_counter() - t0
        reps += 1
    per = t_apply / reps
    return {"value": round(2 * n * n / per / 1e6, 3), "unit": "Munknowns/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle 2-D FFT apply (scipy.fft, 1 worker, FP64, P = {2 * n}) of 1 rhs at n={n}, "
                      f"{reps} repetitions, {per:.2f} s each; symbol setup {t_setup:.1f} s untimed"}


def solve_section(n: int, ndirs: int, binding, I, torch, train_media: int = 4, train_steps: int = 1500,
                  exact_iters: bool = True, host_factor_chosen: bool = False, host_factor_plain: bool = False):
    """Per-rhs time to a 1e-8 relative residual: plain FP64 against the chosen form.

    Plain: class stencils (the paper's 27 fits), complex128 factor, FP64
    apply, one rhs at a time.  Chosen: learned per-point stencils (network
    trained here on exact per-point fits of other seeded media, exact fit
    where it is not accepted), complex64 factor, FP32 apply inside the FP64
    outer FGMRES, ndirs Fibonacci directions x 2 polarisations solved as one
    block with the autotuned apply.  Both factor and solve S in HBM on the
    GPU; optionally the plain path and the chosen block are also timed with
    the host factor.  Set-up (training, fits, factorisations) is timed apart.
    """
    import numpy as np
    dev = torch.device("cuda:0")
    k = I.wavenumber_for(n)
    nb = 2 * ndirs
    interior = [(a * n + b) * n + c for a in range(1, n - 1) for b in range(1, n - 1) for c in range(1, n - 1)]

    # --- set-up: train the stencil network on other media
    t0 = time.perf_counter()
    net = binding.Mlp(binding.Mlp.flat(_init_params(7)))
    for seed in range(1000, 1000 + train_media):
        pt = binding.Plan(n, k, torch.from_numpy(I.medium_bumps(n, seed)).to(dev))
        net.add_samples(pt, interior)
        pt.close()
    torch.cuda.synchronize()
    t_samples = time.perf_counter() - t0
    _progress(f"training samples: {t_samples:.1f} s")
    t0 = time.perf_counter()
    loss = net.train(train_steps, batch=1024, lr=1e-3, seed=0)
    t_train = time.perf_counter() - t0

    m = torch.from_numpy(I.medium_bumps(n, 3)).to(dev)
    plan = binding.Plan(n, k, m, max_rhs=nb)
    dirs, pols = I.fibonacci_incident_set(ndirs)
    Ei = torch.from_numpy(I.plane_waves(n, k, dirs, pols)).to(dev)
    g = plan.rhs_from_incident(Ei)
    torch.cuda.synchronize()

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    def run(gg, prec):
        return timed(lambda: plan.solve(gg, tol=1e-8, prec=prec))

    # --- plain FP64 path: class stencils, complex128 factor, FP64 apply, one rhs
    t_fit_cls, _ = timed(lambda: plan.stencil_fit(0))
    plain_host = None
    if host_factor_plain:                                 # the factor on host cores
        t_fac_h, _ = timed(plan.factor)
        _progress(f"complex128 host factor: {t_fac_h:.1f} s")
        run(g[:1], "c128")                               # warm-up (kernels, workspaces)
        t_ph, (_, infph, stph) = run(g[:1], "c128")
        _progress(f"plain FP64 solve, host factor: {t_ph:.3f} s")
        plain_host = {"s_per_rhs": round(t_ph, 4), "iters": infph[0]["iters"], "status": stph,
                      "factor_s": round(t_fac_h, 3)}
    t_fac_cls, _ = timed(lambda: plan.factor_gpu("c128"))
    _progress(f"complex128 GPU factor: {t_fac_cls:.2f} s")
    run(g[:1], "c128")                                   # warm-up (kernels, workspaces)
    t_plain, (x1, inf1, st1) = run(g[:1], "c128")
    _progress(f"plain FP64 solve: {t_plain:.3f} s")
    # the FP32 apply alone: class stencils, complex128 factor, one rhs
    t_f32one, (_, inf32, st32) = run(g[:1], "mixed")
    _progress(f"FP32-apply single-rhs solve: {t_f32one:.3f} s")
    # --- chosen path: exact per-point fit (for its time and, optionally, its
    # iterations), then the learned fit
    t_fit_pt, _ = timed(lambda: plan.stencil_fit(1))
    exact = None
    if exact_iters:
        plan.factor_gpu("c64")
        _, (_, infx, stx) = run(g[:1], "mixed")
        exact = {"iters": infx[0]["iters"], "status": stx}
        _progress(f"exact per-point stencils: {infx[0]['iters']} iterations")
    t_fit_lrn, nfb = timed(lambda: plan.stencil_fit_learned(net))
    _progress(f"learned fit: {nfb} of {len(interior)} points fell back")
    tune = plan.tune(nb, "mixed")                         # launch choice of the batched apply
    host_chosen = None
    if host_factor_chosen:                                # the same block solve with the host factor
        t_fac_lrn_h, _ = timed(lambda: plan.factor("c64"))
        _progress(f"complex64 host factor: {t_fac_lrn_h:.1f} s")
        t_mixed_h, (_, infh, sth) = run(g, "mixed")
        _progress(f"block mixed solve of {nb}, host factor: {t_mixed_h:.3f} s")
        host_chosen = {"s_per_rhs": round(t_mixed_h / nb, 4), "iters_max": max(i["iters"] for i in infh),
                       "status": sth, "factor_s": round(t_fac_lrn_h, 3),
                       "host_s": round(max(i["t_host"] for i in infh), 4)}
    t_fac_lrn, _ = timed(lambda: plan.factor_gpu("c64"))          # complex64 factor in HBM
    _progress(f"complex64 GPU factor: {t_fac_lrn:.2f} s")
    # the first block call allocates the block's Krylov basis and solve
    # workspaces (about 25 GB at n = 64, 64 rhs); the reported time is the
    # repeated solve, the first call's is recorded beside it
    t_first, _ = run(g, "mixed")
    t_mixed, (xb, infb, stb) = run(g, "mixed")
    _progress(f"block mixed solve of {nb}: {t_mixed:.3f} s")
    # residuals re-measured with the FP64 apply: r = g - A x
    r = torch.empty_like(g)
    plan.apply(xb, r, prec="c128")
    rel = (torch.linalg.vector_norm((g - r).reshape(nb, -1), dim=1) /
           torch.linalg.vector_norm(g.reshape(nb, -1), dim=1)).max().item()
    plan.close()
    net.close()
    return {
        "n": n, "unknowns_per_rhs": 3 * n ** 3, "nrhs_batched": nb,
        "plain_fp64_s_per_rhs": round(t_plain, 4), "plain_iters": inf1[0]["iters"],
        "chosen_s_per_rhs": round(t_mixed / nb, 4),
        "chosen_first_call_s_per_rhs": round(t_first / nb, 4),
        "chosen_iters_max": max(i["iters"] for i in infb),
        "chosen_max_rel_resid_fp64": float(f"{rel:.3e}"),
        "status": [st1, st32, stb],
        "plain_with_host_factor": plain_host,
        "speedup_per_rhs": round(t_plain / (t_mixed / nb), 2),
        "fp32_apply_single_rhs_s": round(t_f32one, 4), "fp32_apply_single_rhs_iters": inf32[0]["iters"],
        "exact_point_stencils_iters": exact["iters"] if exact else None,
        "chosen_with_host_factor": host_chosen,
        "learned_fallback_points": int(nfb), "interior_points": len(interior),
        "setup_s": {"samples": round(t_samples, 3), "train": round(t_train, 3),
                    "train_loss_first_last": [round(float(loss[0]), 4), round(float(np.mean(loss[-20:])), 4)],
                    "class_fit": round(t_fit_cls, 3), "point_fit_exact": round(t_fit_pt, 3),
                    "learned_fit": round(t_fit_lrn, 3),
                    "factor_class_c128_gpu": round(t_fac_cls, 3), "factor_learned_c64_gpu": round(t_fac_lrn, 3)},
        "tuned_apply": _tune_choice(tune),
    }


def config4_section(binding, I, torch, n_eval: int = 5, media: int = 200, points: int = 4096,
                    train_steps: int = 8000, n_eval_grid: int = 96):
    """The learned-stencil workload: a network trained on exact per-point fits
    (the medium-weighted fit) of `media` seeded six-bump media at n = 32, 48 and
    64 (seeds 1000, 1001, ...; n cycling), `points` random interior points of
    each, then evaluated on unseen media (seeds 2000, ...) at n = 96 (2.65M
    unknowns) against the exact per-point fit and the paper's class fit.  Each
    of the three stencil sets gets its own complex64 factor of S in HBM and
    the same FGMRES (FP32 apply inside FP64, restart 30, to 1e-8) on one
    seeded plane wave; iterations, fit, factor and solve times are reported,
    with the FP64 residual recomputed by the library's FP64 apply."""
    import numpy as np
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(4)
    net = binding.Mlp(binding.Mlp.flat(_init_params(11)))
    sizes = (32, 48, 64)
    t0 = time.perf_counter()
    for i in range(media):
        n = sizes[i % 3]
        interior = np.array([(a * n + b) * n + c for a in range(1, n - 1) for b in range(1, n - 1)
                             for c in range(1, n - 1)])
        pts = rng.choice(interior, min(points, len(interior)), replace=False)
        pt = binding.Plan(n, I.wavenumber_for(n), torch.from_numpy(I.medium_bumps(n, 1000 + i)).to(dev))
        net.add_samples(pt, pts)
        pt.close()
        if (i + 1) % 50 == 0:
            _progress(f"config 4: samples of {i + 1} media")
    torch.cuda.synchronize()
    t_samples = time.perf_counter() - t0
    t0 = time.perf_counter()
    loss = net.train(train_steps, batch=1024, lr=1e-3, seed=0)
    t_train = time.perf_counter() - t0
    nsamp = net.num_samples()
    _progress(f"config 4: {nsamp} samples in {t_samples:.1f} s, training {t_train:.1f} s")

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t, r

    n = n_eval_grid
    k = I.wavenumber_for(n)
    evals = []
    for e in range(n_eval):
        seed = 2000 + e
        m = torch.from_numpy(I.medium_bumps(n, seed)).to(dev)
        plan = binding.Plan(n, k, m, max_rhs=1)
        d, p = I.random_direction_and_polarisation(seed)
        g = plan.rhs_from_incident(torch.from_numpy(I.plane_waves(n, k, [d], [p])).to(dev))
        row = {"seed": seed}
        for name in ("class", "exact", "learned"):
            if name == "class":
                t_fit, _ = timed(lambda: plan.stencil_fit(0))
                extra = {}
            elif name == "exact":
                t_fit, _ = timed(lambda: plan.stencil_fit(1))
                extra = {}
            else:
                t_fit, nfb = timed(lambda: plan.stencil_fit_learned(net))
                extra = {"fallback_points": int(nfb), "interior_points": (n - 2) ** 3}
            t_fac, _ = timed(lambda: plan.factor_gpu("c64"))
            t_sol, (x, info, st) = timed(lambda: plan.solve(g, tol=1e-8, prec="mixed"))
            r = torch.empty_like(g)
            plan.apply(x, r, prec="c128")
            rel = (torch.linalg.vector_norm(g - r) / torch.linalg.vector_norm(g)).item()
            row[name] = {"iters": info[0]["iters"], "fit_s": round(t_fit, 3), "factor_s": round(t_fac, 2),
                         "solve_s": round(t_sol, 3), "rel_resid_fp64": float(f"{rel:.3e}"), "status": st, **extra}
            _progress(f"config 4: seed {seed} {name}: {info[0]['iters']} iterations, fit {t_fit:.2f} s, "
                      f"factor {t_fac:.1f} s, solve {t_sol:.2f} s")
        plan.close()
        del m, g
        torch.cuda.empty_cache()
        evals.append(row)
    net.close()

    def mean(key, field):
        return round(float(np.mean([r[key][field] for r in evals])), 3)

    return {"train": {"media": media, "grids": list(sizes), "points_per_medium": points,
                      "samples": int(nsamp), "samples_s": round(t_samples, 2),
                      "train_steps": train_steps, "batch": 1024, "train_s": round(t_train, 2),
                      "loss_first_last": [round(float(loss[0]), 4), round(float(np.mean(loss[-50:])), 4)]},
            "eval_n": n, "eval_unknowns": 3 * n ** 3, "eval": evals,
            "mean": {v: {"iters": mean(v, "iters"), "fit_s": mean(v, "fit_s"), "solve_s": mean(v, "solve_s")}
                     for v in ("class", "exact", "learned")},
            "learned_fallback_fraction": round(float(np.mean([r["learned"]["fallback_points"] /
                                                              r["learned"]["interior_points"] for r in evals])), 4)}


def solve_config1(n: int, binding, I, torch):
    """The plain FP64 path on the GPU for the oracle's solve baseline: the same
    medium and plane wave, class stencils, complex128 factor of S in HBM, FP64
    apply, FGMRES(30) to 1e-8, one rhs (median of 5 solves after a warm-up)."""
    dev = torch.device("cuda:0")
    k = I.wavenumber_for(n)
    m = I.medium_single_bump(n, 0) if n == 16 else I.medium_bumps(n, 1)
    d, p = I.random_direction_and_polarisation(0)
    plan = binding.Plan(n, k, torch.from_numpy(m).to(dev), max_rhs=1)
    g = plan.rhs_from_incident(torch.from_numpy(I.plane_waves(n, k, [d], [p])).to(dev))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.stencil_fit(0)
    plan.factor_gpu("c128")
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    plan.solve(g, tol=1e-8, prec="c128")
    ts = []
    for _ in range(5):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, info, st = plan.solve(g, tol=1e-8, prec="c128")
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    plan.close()
    ts.sort()
    return {"n": n, "plain_fp64_s_per_rhs": round(ts[2], 5), "iters": info[0]["iters"],
            "rel_resid": info[0]["rel_resid"], "status": st, "setup_s": round(t_setup, 3)}


def _progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _init_params(seed: int):
    """He-normal weights, zero biases, in the network's flat layout (250-256-256-468)."""
    import numpy as np
    g = np.random.default_rng(seed)
    dims = [(250, 256), (256, 256), (256, 468)]
    p = {}
    for i, (a, b) in enumerate(dims, 1):
        p[f"W{i}"] = g.standard_normal((a, b)) * np.sqrt(2.0 / a)
        p[f"b{i}"] = np.zeros(b)
    return p


def _tune_choice(t: dict) -> dict:
    return {k: t[k] for k in ("chunk", "kmul_w", "half_runs", "persist", "ms_per_rhs", "ms_default_per_rhs")}


def apply_192(binding, I, torch, steps: int, B: int = 8):
    """The apply at n = 192 (padded 384^3 FFTs), FP32, 8 rhs: throughput and pass rates."""
    import numpy as np
    dev = torch.device("cuda:0")
    n = 192
    m = torch.from_numpy(I.medium_bumps(n, 3)).to(dev)
    plan = binding.Plan(n, I.wavenumber_for(n), m, max_rhs=B)
    P = plan.P
    g = torch.Generator(device=dev).manual_seed(99)
    x = torch.randn((B, 3, n, n, n), dtype=torch.complex64, device=dev, generator=g)
    y = torch.empty_like(x)
    tune = plan.tune(B, "c64")                # launch choices (set-up, outside the timed region)
    for _ in range(3):
        plan.apply(x, y, prec="c64")
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    reps = max(5, steps // 5)
    e0.record()
    for _ in range(reps):
        plan.apply(x, y, prec="c64")
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    pms = np.zeros(5)
    for _ in range(5):
        pms += np.array(plan.apply_timed(x, y, prec="c64"))
    pms /= 5
    pb = pass_bytes(n, P, B, 8, 8)
    plan.close()
    del x, y
    torch.cuda.empty_cache()
    return {"n": n, "fft_size": P, "nrhs": B, "tuned": _tune_choice(tune), "ms_per_apply": round(ms, 3),
            "Munknowns_per_s": round(B * 3 * n ** 3 / (ms * 1e-3) / 1e6, 1),
            "whole_GBps": round(sum(pb) / (ms * 1e-3) / 1e9, 1),
            "pass_ms": [round(v, 4) for v in pms],
            "pass_GBps": [round(b / (t * 1e-3) / 1e9, 1) for b, t in zip(pb, pms)]}


def pass_bytes_2d(n: int, P: int, H: int, B: int, s: int, s_io: int) -> list[float]:
    """Algorithmic HBM bytes of the three passes of the 2-D apply for B rhs:
    intermediates of s bytes per complex, fields of s_io bytes per complex.
    A: x, m, p read, the three row-transformed fields written ([B][3][n][P]);
    B: those read, the symbol quadrant read once, two products written;
    C: the products read, x read, y written."""
    nn = n * n
    a = B * 2 * nn * s_io + 3 * nn * s + B * 3 * n * P * s
    b = B * 3 * n * P * s + 3 * H * H * s + B * 2 * n * P * s
    c = B * 2 * n * P * s + 2 * B * 2 * nn * s_io
    return [a, b, c]


def two_d_section(binding, I, torch, steps: int, n: int = 959, B: int = 8, solve_n: int = 959):
    """The 2-D variant at the paper's largest 2-D grid (n = 959, P = 1944,
    six points per wavelength): apply throughput, pass times and the
    roofline of the dominant pass; and the paper's 2-D lens example solved
    with its settings (class stencils, complex128 factor in HBM, GMRES(20)
    to 1e-6)."""
    import numpy as np
    dev = torch.device("cuda:0")
    k = I.paper_wavenumber(n)
    m = torch.from_numpy(I.medium2_perturbed_square(n, 3)).to(dev)
    plan = binding.Plan2(n, k, m, max_rhs=B)
    P, H = plan.P, plan.P // 2 + 1
    g = torch.Generator(device=dev).manual_seed(7)
    x64 = torch.randn((B, 2, n, n), dtype=torch.complex128, device=dev, generator=g)
    x32 = x64.to(torch.complex64)
    y32, y64 = torch.empty_like(x32), torch.empty_like(x64)

    def timed(prec, x, y, reps):
        for _ in range(3):
            plan.apply(x, y, prec=prec)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            plan.apply(x, y, prec=prec)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    reps = max(5, steps)
    ms32 = timed("c64", x32, y32, reps)
    ms64 = timed("c128", x64, y64, max(5, reps // 2))
    msmx = timed("mixed", x64, y64, max(5, reps // 2))
    pms = np.zeros(3)
    for _ in range(10):
        pms += np.array(plan.apply_timed(x32, y32, prec="c64"))
    pms /= 10
    pb = pass_bytes_2d(n, P, H, B, 8, 8)
    dom = int(np.argmax(pms))
    achieved = pb[dom] / (pms[dom] * 1e-3) / 1e9
    unknowns = B * 2 * n * n
    plan.close()
    del x64, x32, y32, y64
    torch.cuda.empty_cache()
    out = {"workload": f"2-D apply, n={n} (P={P}), {B} rhs, FP32 FFTs", "n": n, "fft_size": P, "nrhs": B,
           "Munknowns_per_s": round(unknowns / (ms32 * 1e-3) / 1e6, 1), "ms_per_apply": round(ms32, 4),
           "c128_Munknowns_per_s": round(unknowns / (ms64 * 1e-3) / 1e6, 1),
           "mixed_Munknowns_per_s": round(unknowns / (msmx * 1e-3) / 1e6, 1),
           "pass_ms": [round(v, 4) for v in pms],
           "pass_GBps": [round(b / (t * 1e-3) / 1e9, 1) for b, t in zip(pb, pms)],
           "whole_GBps": round(sum(pb) / (ms32 * 1e-3) / 1e9, 1),
           "roofline": {"bound": "hbm", "kernel": ["pass_a_kernel", "pass_b_kernel", "pass_c_kernel"][dom],
                        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": measured_traffic(n, B, "c64", MEASURED_TRAFFIC_2D) if dom == 1 else None,
                        "algorithmic_bytes": round(pb[dom])}}
    if solve_n:
        import time
        ks = I.paper_wavenumber(solve_n)
        ms_ = torch.from_numpy(I.medium2_lens(solve_n)).to(dev)
        plan = binding.Plan2(solve_n, ks, ms_, max_rhs=1)
        gg = plan.rhs_from_incident(torch.from_numpy(I.paper_incident2(solve_n, ks)).to(dev))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.stencil_fit()
        t_fac = plan.factor_gpu("c128")
        t_setup = time.perf_counter() - t0
        v = torch.randn_like(gg)
        z = torch.empty_like(gg)
        plan.precond(v, z)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            plan.precond(v, z)
        torch.cuda.synchronize()
        t_app = (time.perf_counter() - t0) / 3
        plan.solve(gg, tol=1e-6, restart=20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info, st = plan.solve(gg, tol=1e-6, restart=20)
        torch.cuda.synchronize()
        t_sol = time.perf_counter() - t0
        # many incident directions at once: a lockstep block of FGMRES, one
        # GPU solve of S for the whole block per Arnoldi step
        nd = 16
        d, pol = I.circle_incident_set2(nd)
        gb = plan.rhs_from_incident(torch.from_numpy(I.plane_waves2(solve_n, ks, d, pol)).to(dev))
        plan.solve(gb, tol=1e-6, restart=20)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        xb, infob, stb = plan.solve(gb, tol=1e-6, restart=20)
        torch.cuda.synchronize()
        t_blk = time.perf_counter() - t0
        plan.close()
        out["paper_lens_solve"] = {"n": solve_n, "k_over_2pi": round(ks / (2 * math.pi), 3), "N": 2 * solve_n ** 2,
                                   "T_setup": round(t_setup, 3), "T_factor": round(t_fac, 3),
                                   "T_apply": round(t_app, 4), "N_iter": info[0]["iters"],
                                   "T_solve": round(t_sol, 3), "rel_resid": info[0]["rel_resid"], "status": st,
                                   "block_rhs": nd, "block_s_per_rhs": round(t_blk / nd, 4),
                                   "block_iters_max": max(i["iters"] for i in infob),
                                   "block_max_rel_resid": max(i["rel_resid"] for i in infob), "block_status": stb}
    return out


def hbm_copy_gbps(torch, binding, gib: float = 2.0):
    """Device-to-device copy bandwidth (read + write bytes / time): torch's copy
    and the library's streaming copy (ls_hbm_copy), the achievable ceiling."""
    n = int(gib * (1 << 30)) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda:0").fill_(1.0)
    b = torch.empty_like(a)
    out = []
    for fn in (lambda: b.copy_(a), lambda: binding.hbm_copy(b, a, n * 4)):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out.append(round(2 * a.numel() * 4 / (e0.elapsed_time(e1) / 5 * 1e-3) / 1e9, 1))
    del a, b
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--nrhs", type=int, default=8)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--config4", type=int, default=0,
                    help="learned-stencil workload: unseen media evaluated at 96^3 (0: skip; ~70 s each)")
    ap.add_argument("--config4-media", type=int, default=200, help="training media of the learned workload")
    ap.add_argument("--cpu-n", type=int, default=128)
    ap.add_argument("--cpu-solve-n", type=int, default=16,
                    help="grid of the oracle's per-rhs solve baseline (0: skip; 32 takes ~7 min of set-up)")
    ap.add_argument("--no-n192", dest="n192", action="store_false", help="skip the 192^3 apply line")
    ap.add_argument("--two-d-n", type=int, default=959, help="grid of the 2-D variant's apply line (0: skip)")
    ap.add_argument("--two-d-solve-n", type=int, default=959, help="grid of the 2-D lens solve (0: skip)")
    ap.add_argument("--solve-n", type=int, default=64, help="grid of the per-rhs solve section (0: skip)")
    ap.add_argument("--solve-dirs", type=int, default=32, help="incident directions (2 polarisations each)")
    ap.add_argument("--solve-exact", type=int, default=-1,
                    help="also solve with the exact per-point stencils (1/0; default: when n <= 48)")
    ap.add_argument("--solve-host-factor", type=int, default=-1,
                    help="also time the plain path and the chosen block with host factors (1/0; default: n <= 32)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); the path shards by "
              "right-hand side, each GPU running this single-GPU path on its share", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1804_02297_amd import binding
    from paper_1804_02297_amd import inputs as I

    binding.load()
    dev = torch.device("cuda:0")
    n, B = args.n, args.nrhs
    k = I.wavenumber_for(n)
    m = torch.from_numpy(I.medium_bumps(n, 3)).to(dev)
    plan = binding.Plan(n, k, m, max_rhs=B)
    P = plan.P
    g = torch.Generator(device=dev).manual_seed(1234)
    x64 = torch.randn((B, 3, n, n, n), dtype=torch.complex128, device=dev, generator=g)
    x32 = x64.to(torch.complex64)
    y32 = torch.empty_like(x32)
    y64 = torch.empty_like(x64)
    # launch choices of the FP32 apply from the autotuner (set-up, untimed)
    tune32 = plan.tune(B, "c64")
    torch.cuda.synchronize()

    def timed(prec, x, y, steps, warmup):
        for _ in range(warmup):
            plan.apply(x, y, prec=prec)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            plan.apply(x, y, prec=prec)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return e0.elapsed_time(e1) / steps, wall

    ms32, wall32 = timed("c64", x32, y32, args.steps, args.warmup)
    # per-pass times over the same number of steps
    pms = np.zeros(5)
    for _ in range(max(3, min(args.steps, 20))):
        pms += np.array(plan.apply_timed(x32, y32, prec="c64"))
    pms /= max(3, min(args.steps, 20))
    ms64, _ = timed("c128", x64, y64, max(5, args.steps // 2), 2)
    msmx, _ = timed("mixed", x64, y64, max(5, args.steps // 2), 2)
    # the paper's own 3x4 form on the same plan (four forward transforms, three inverse)
    plan.set_form("paper")
    ms_pf, _ = timed("c64", x32, y32, max(5, args.steps // 2), 2)
    ms_pf64, _ = timed("c128", x64, y64, max(5, args.steps // 4), 1)
    plan.set_form("dyadic")

    unknowns = B * 3 * n ** 3
    value = unknowns / (ms32 * 1e-3) / 1e6
    pb = pass_bytes(n, P, B, 8, 8)
    dom = int(np.argmax(pms))
    achieved = pb[dom] / (pms[dom] * 1e-3) / 1e9
    whole = sum(pb) / (ms32 * 1e-3) / 1e9

    out = {
        "metric": "Munknowns/s of LS apply at 128^3",
        "value": round(value, 1),
        "unit": "Munknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64",
        "data": "synthetic: seeded sum-of-6-Gaussians contrast, random complex fields",
        "config": {"workload": f"LS apply, n={n} (P={P}), {B} rhs, FP32 FFTs",
                   "n": n, "fft_size": P, "nrhs": B, "unknowns_per_rhs": 3 * n ** 3},
        "tuned": _tune_choice(tune32),
        "roofline": {"bound": "hbm", "kernel": KERNEL_NAMES[dom], "pass": PASS_NAMES[dom],
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(n, B, "c64") if dom == 2 else None,
                     "algorithmic_bytes": round(pb[dom])},
        "apply_whole_GBps": round(whole, 1),
        "apply_whole_frac": round(whole / HBM_PEAK_GBS, 4),
        "pass_ms": [round(v, 4) for v in pms],
        "pass_GBps": [round(b / (t * 1e-3) / 1e9, 1) for b, t in zip(pb, pms)],
        "c128_Munknowns_per_s": round(unknowns / (ms64 * 1e-3) / 1e6, 1),
        "mixed_Munknowns_per_s": round(unknowns / (msmx * 1e-3) / 1e6, 1),
        "paper_form_Munknowns_per_s": round(unknowns / (ms_pf * 1e-3) / 1e6, 1),
        "paper_form_c128_Munknowns_per_s": round(unknowns / (ms_pf64 * 1e-3) / 1e6, 1),
        "wall_s_timed": round(wall32, 3),
    }
    if args.n192:
        out["apply_192"] = apply_192(binding, I, torch, args.steps)
    if args.two_d_n:
        _progress("2-D variant")
        out["two_d"] = two_d_section(binding, I, torch, args.steps, n=args.two_d_n, solve_n=args.two_d_solve_n)
    torch_copy, stream_copy = hbm_copy_gbps(torch, binding)
    out["hbm_copy_GBps"] = torch_copy
    out["hbm_stream_copy_GBps"] = stream_copy
    out["roofline"]["copy_ceiling_GBps"] = stream_copy
    out["apply_whole_frac_of_copy"] = round(whole / stream_copy, 4)
    if args.solve_n:
        ex = (args.solve_n <= 48) if args.solve_exact < 0 else bool(args.solve_exact)
        hf = (args.solve_n <= 32) if args.solve_host_factor < 0 else bool(args.solve_host_factor)
        out["solve"] = solve_section(args.solve_n, args.solve_dirs, binding, I, torch, exact_iters=ex,
                                     host_factor_chosen=hf, host_factor_plain=hf)
    if args.config4:
        out["config4"] = config4_section(binding, I, torch, n_eval=args.config4, media=args.config4_media)
    if args.cpu_solve_n and not args.no_cpu:
        out["solve_config1"] = solve_config1(args.cpu_solve_n, binding, I, torch)
    if not args.no_cpu:
        _progress("CPU oracle baselines")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n)
        if args.cpu_solve_n:
            out["cpu_baseline"]["solve"] = cpu_baseline_solve(args.cpu_solve_n)
            if "solve_config1" in out:
                out["cpu_baseline"]["solve"]["gpu_over_cpu_per_rhs"] = round(
                    out["cpu_baseline"]["solve"]["value"] / out["solve_config1"]["plain_fp64_s_per_rhs"], 1)
        if args.two_d_n:
            out["cpu_baseline"]["two_d"] = cpu_baseline_2d(args.two_d_n)
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
