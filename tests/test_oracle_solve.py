"""Pins of the oracle's sparse rows, preconditioner and FGMRES.

* Eq. (11)/(12): (Q A - S) vanishes on every row's own neighbourhood, so Q A
  and S differ only by the dropped non-local term alpha^H M diag(m);
* m = 0: S == Q exactly, P^-1 = S^-1 Q = I, FGMRES converges in one step;
* gauge invariance: S^-1 Q is unchanged by alpha -> alpha X;
* FGMRES against numpy.linalg.solve on dense tiny systems; an exact
  preconditioner converges in one iteration;
* reciprocity of total fields (diag(m) (I + K diag(m))^-1 is symmetric);
* the paper's qualitative claim (Section 4): preconditioned iterations stay
  below ten at six points per wavelength, GMRES(20), tolerance 1e-6.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import fgmres as fg
from oracle import operator as op
from oracle import sparse as sp
from oracle import stencil as st
from paper_1804_02297_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _setup(n, seed=0, amp=-0.2):
    k = I.wavenumber_for(n)
    m = I.medium_single_bump(n, seed, amplitude=amp)
    al, be, _ = st.fit_all_classes(n, k)
    S, Q = sp.assemble(n, m, al, be)
    return k, m, al, be, S, Q


def test_local_part_of_QA_equals_S():
    n = 6
    k, m, al, be, S, Q = _setup(n)
    A = op.dense_matrix(n, k, m)
    D = (Q @ A) - S.toarray()
    mask = (S != 0).toarray() | (Q != 0).toarray()
    assert np.abs(D[mask]).max() <= 1e-13 * np.abs(S.toarray()).max()
    # the dropped part is small compared with the kept part
    assert np.linalg.norm(D) < 0.2 * np.linalg.norm(S.toarray())


def test_zero_contrast():
    n = 5
    k = I.wavenumber_for(n)
    m = np.zeros((n, n, n), complex)
    al, be, _ = st.fit_all_classes(n, k)
    S, Q = sp.assemble(n, m, al, be)
    assert (S != Q).nnz == 0
    P = sp.Preconditioner(S, Q)
    g = I.random_field(1, n, 1)[0]
    assert np.allclose(P(g), g, rtol=0, atol=1e-12)
    x, info = fg.fgmres(lambda v: op.apply_fft(n, k, m, v), g, P, tol=1e-10)
    assert info["iters"] == 1
    assert np.abs(x - g).max() <= 1e-12


def test_gauge_invariance():
    n = 5
    k, m, al, be, S, Q = _setup(n, amp=-0.3)
    rng = np.random.default_rng(0)
    al2, be2 = [], []
    for a, b in zip(al, be):
        X = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3)) + 3 * np.eye(3)
        al2.append(a @ X)
        be2.append(b @ X)
    S2, Q2 = sp.assemble(n, m, al2, be2)
    v = I.random_field(1, n, 3)[0]
    z1 = sp.Preconditioner(S, Q)(v)
    z2 = sp.Preconditioner(S2, Q2)(v)
    assert np.abs(z1 - z2).max() <= 1e-10 * np.abs(z1).max()


@pytest.mark.parametrize("n", [3, 4])
def test_fgmres_matches_dense_solve(n):
    k = I.wavenumber_for(n)
    m = I.medium_random_complex(n, 7, scale=0.2)
    A = op.dense_matrix(n, k, m)
    g = I.random_field(1, n, 8)[0]
    xref = np.linalg.solve(A, g.reshape(-1))
    x, info = fg.fgmres(lambda v: op.apply_fft(n, k, m, v), g, None, tol=1e-12, restart=5)
    kappa = np.linalg.cond(A)
    assert np.abs(x.reshape(-1) - xref).max() <= kappa * 1e-11 * np.abs(xref).max()
    assert info["rel_resid"] <= 1e-12
    assert info["restarts"] >= 1
    # exact preconditioner: one iteration
    Ainv = np.linalg.inv(A)
    x2, info2 = fg.fgmres(lambda v: op.apply_fft(n, k, m, v), g,
                          lambda v: (Ainv @ v.reshape(-1)).reshape(v.shape), tol=1e-10)
    assert info2["iters"] == 1


def test_preconditioned_solve_and_reciprocity():
    n = 8
    k, m, al, be, S, Q = _setup(n, amp=-0.3)
    P = sp.Preconditioner(S, Q)
    Kh = op.kernel_symbol(n, k)
    A = lambda v: op.apply_fft(n, k, m, v, Kh)
    d1, d2 = np.array([1.0, 0, 0]), np.array([0, 0.6, 0.8])
    p1, p2 = np.array([0, 0, 1.0]), np.array([1.0, 0, 0])
    E = I.plane_waves(n, k, [d1, d2], [p1, p2])
    tot = []
    its = []
    for r in range(2):
        g = op.rhs_from_incident(n, k, m, E[r:r + 1], Kh)[0]
        x, info = fg.fgmres(A, g, P, tol=1e-10)
        assert info["rel_resid"] <= 1e-10
        tot.append(E[r] + x)
        its.append(info["iters"])
        _, info0 = fg.fgmres(A, g, None, tol=1e-10)
        assert info["iters"] < info0["iters"]
    lhs = np.sum(E[0] * m[None] * tot[1])
    rhs = np.sum(E[1] * m[None] * tot[0])
    assert abs(lhs - rhs) <= 1e-8 * abs(lhs)


@pytest.mark.slow
def test_paper_iteration_claim_three_d():
    """Section 4: below ten iterations at 6 points per wavelength, GMRES(20), tol 1e-6."""
    with open(os.path.join(GOLDEN, "paper_tables_3d.json")) as f:
        gold = json.load(f)
    assert max(r["N_iter"] for r in gold["rows"]) < gold["claim_max_iters"]
    n = 11
    k = 2 * math.pi * (n + 1) / 6.0         # six points per wavelength with h = 1/(n+1)
    m = I.medium_bumps(n, 5)
    al, be, _ = st.fit_all_classes(n, k)
    S, Q = sp.assemble(n, m, al, be)
    P = sp.Preconditioner(S, Q)
    Ei = I.plane_waves(n, k, [[1.0, 0, 0]], [[0, 0, 1.0]])
    g = op.rhs_from_incident(n, k, m, Ei)[0]
    x, info = fg.fgmres(lambda v: op.apply_fft(n, k, m, v), g, P, tol=1e-6, restart=20)
    assert info["iters"] < gold["claim_max_iters"]
