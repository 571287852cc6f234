"""Right-preconditioned flexible GMRES in FP64 (oracle).  TEST INFRASTRUCTURE ONLY.

Paper: the preconditioner is combined with standard GMRES (end of Section 3.1,
Section 4: restart 20, relative residual 1e-6).  Reading taken: right
preconditioning, so the residual that is monitored is the unpreconditioned
||g - A x|| / ||g||; x0 = 0; modified Gram-Schmidt Arnoldi with complex
Givens rotations; flexible form (the preconditioned vectors z_j are stored)
so that a preconditioner that changes between iterations is allowed.  At
every restart the true residual is recomputed with the FP64 apply; the solve
ends only when that true residual meets tol (or maxit is reached).

Pins: tiny dense problems against numpy.linalg.solve; P = exact inverse
converges in one iteration; m = 0 gives x = g after one iteration.
"""
from __future__ import annotations

import numpy as np


def _givens(a: complex, b: complex):
    """Real c, complex s with [c s; -conj(s) c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, 1.0 + 0.0j
    den = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    c = abs(a) / den
    s = (a / abs(a)) * np.conj(b) / den
    return c, s


def fgmres(apply_A, g: np.ndarray, precond=None, tol: float = 1e-8, restart: int = 30,
           maxit: int = 1000):
    """Solve A x = g.  Returns (x, info), info = dict(iters, restarts, rel_resid, history)."""
    if precond is None:
        def precond(v):
            return v
    shp = g.shape
    gv = g.reshape(-1).astype(np.complex128)
    gnorm = np.linalg.norm(gv)
    x = np.zeros_like(gv)
    hist = []
    if gnorm == 0.0:
        return x.reshape(shp), dict(iters=0, restarts=0, rel_resid=0.0, history=hist)
    total = 0
    restarts = 0
    while True:
        r = gv - apply_A(x.reshape(shp)).reshape(-1)
        beta = np.linalg.norm(r)
        rel = beta / gnorm
        if rel <= tol or total >= maxit:
            return x.reshape(shp), dict(iters=total, restarts=restarts, rel_resid=rel, history=hist)
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart)
        sn = np.zeros(restart, dtype=np.complex128)
        e = np.zeros(restart + 1, dtype=np.complex128)
        e[0] = beta
        j_used = 0
        for j in range(restart):
            z = precond(V[j].reshape(shp)).reshape(-1)
            Z.append(z)
            w = apply_A(z.reshape(shp)).reshape(-1)
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            for i in range(j):                          # earlier rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            e[j + 1] = -np.conj(sn[j]) * e[j]
            e[j] = cs[j] * e[j]
            total += 1
            j_used = j + 1
            hist.append(abs(e[j + 1]) / gnorm)
            if hist[-1] <= tol or total >= maxit or hn == 0.0:
                break
            V.append(w / hn)
        y = np.linalg.solve(np.triu(H[:j_used, :j_used]), e[:j_used])
        for i in range(j_used):
            x = x + y[i] * Z[i]
        restarts += 1
