"""Sparse rows S, Q and the preconditioner S^-1 Q (oracle, FP64).
TEST INFRASTRUCTURE ONLY.

Paper: Eq. (11) (the three local rows per point), Eq. (12) (beta), end of
Section 3.1 (assemble all rows, replace the approximate sign with equality,
solve the sparse system as the preconditioner), Section 3.3 (sparse direct
solve).  For point i in class kappa and each neighbour offset a in tau:

  Q[(r, i), (c, i+a)] = conj(alpha[(a, c), r])
  S[(r, i), (c, i+a)] = conj(alpha[(a, c), r]) + conj(beta[(a, c), r]) m_{i+a}

so that S E = Q g are the rows alpha^H E_tau + beta^H diag(m)_tau E_tau =
alpha^H g_tau of Eq. (11).  Unknowns and rows are ordered [c, i1, i2, i3]
like the fields.  The preconditioner is P^-1 v = S^-1 (Q v), with SciPy's
SuperLU as the sparse direct solver (the paper uses nested dissection; any
exact sparse solver gives the same P^-1).

Pins: m = 0 gives S = Q A restricted to the local rows exactly... (see
tests/test_oracle_sparse.py: S == Q when m = 0 and P^-1 A = I for m = 0).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse
import scipy.sparse.linalg

from .stencil import class_of_point, tau_offsets


def assemble(n: int, m: np.ndarray, alphas, betas):
    """S and Q as CSR matrices (3n^3 x 3n^3) from per-class stencils."""
    return assemble_pointwise(n, m, lambda i1, i2, i3, kappa: (alphas[kappa], betas[kappa]))


def assemble_pointwise(n: int, m: np.ndarray, stencil_of):
    """S and Q from a per-point stencil callback stencil_of(i1, i2, i3, kappa) -> (alpha, beta).

    i1, i2, i3 are 0-based grid indices.
    """
    N = n ** 3
    rows, cols, sv, qv = [], [], [], []
    mm = np.asarray(m, dtype=np.complex128)
    for i1 in range(n):
        for i2 in range(n):
            for i3 in range(n):
                kappa = class_of_point(i1 + 1, i2 + 1, i3 + 1, n)
                alpha, beta = stencil_of(i1, i2, i3, kappa)
                tau = tau_offsets(kappa)
                pi = (i1 * n + i2) * n + i3
                for t, a in enumerate(tau):
                    j1, j2, j3 = i1 + a[0], i2 + a[1], i3 + a[2]
                    pj = (j1 * n + j2) * n + j3
                    mj = mm[j1, j2, j3]
                    for r in range(3):
                        for c in range(3):
                            qa = np.conj(alpha[3 * t + c, r])
                            rows.append(r * N + pi)
                            cols.append(c * N + pj)
                            qv.append(qa)
                            sv.append(qa + np.conj(beta[3 * t + c, r]) * mj)
    shape = (3 * N, 3 * N)
    S = scipy.sparse.csr_matrix((np.array(sv), (rows, cols)), shape=shape)
    Q = scipy.sparse.csr_matrix((np.array(qv), (rows, cols)), shape=shape)
    return S, Q


class Preconditioner:
    """P^-1 v = S^-1 (Q v) with an exact sparse LU of S."""

    def __init__(self, S, Q):
        self.Q = Q.tocsr()
        self.lu = scipy.sparse.linalg.splu(S.tocsc())

    def __call__(self, v: np.ndarray) -> np.ndarray:
        shp = v.shape
        return self.lu.solve(self.Q @ v.reshape(-1)).reshape(shp)
