"""Pins of the oracle's paper form (Section 2, the 3x4 discrete equations).

Each pin checks the oracle against something other than its own formula: a
literal double sum, a finite difference of G, a quadrature over the ball,
the second-order convergence of the central differences to an analytic
gradient, the identity at m = 0, and the approach of this form's solution
to the dyadic form's as the grid is refined (both discretise the same
continuous equation).
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.sparse.linalg as spla

from oracle import kernel as okr
from oracle import operator as oop
from oracle import paper_form as opf
from paper_1804_02297_amd import inputs as I


@pytest.mark.parametrize("n", [3, 4, 5])
def test_fft_apply_equals_double_sum(n):
    g = np.random.default_rng(n)
    m = 0.2 * (g.standard_normal((n, n, n)) + 1j * g.standard_normal((n, n, n)))
    x = g.standard_normal((3, n, n, n)) + 1j * g.standard_normal((3, n, n, n))
    k = 2 * math.pi * 1.3
    a = opf.apply_fft_paper(n, k, m, x)
    b = opf.apply_dense_paper(n, k, m, x)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_gradient_of_G_matches_finite_differences():
    k = 7.0
    pts = np.array([[0.3, -0.2, 0.1], [0.05, 0.4, -0.3], [-0.6, 0.0, 0.2]])
    d = 1e-6
    for x in pts:
        num = np.array([(okr.helmholtz_G(np.linalg.norm(x + d * e), k) - okr.helmholtz_G(np.linalg.norm(x - d * e), k))
                        / (2 * d) for e in np.eye(3)])
        assert np.abs(opf.dG(x, k) - num).max() <= 1e-7 * np.abs(num).max()


@pytest.mark.parametrize("k,h", [(5.0, 0.05), (20.0, 1 / 30), (60.0, 1 / 60)])
def test_self_weight_is_the_ball_integral(k, h):
    a = h * (3 / (4 * math.pi)) ** (1 / 3)
    re = scipy.integrate.quad(lambda r: r * math.cos(k * r), 0, a, epsabs=1e-16, epsrel=1e-13)[0]
    im = scipy.integrate.quad(lambda r: r * math.sin(k * r), 0, a, epsabs=1e-16, epsrel=1e-13)[0]
    # int_ball e^{ikr}/(4 pi r) dV = int_0^a r e^{ikr} dr
    assert abs(opf.ball_integral_G(k, h) - (re + 1j * im)) <= 1e-12 * abs(re + 1j * im)
    # volume check of the equal-volume ball: (4/3) pi a^3 = h^3
    assert abs(4 / 3 * math.pi * a ** 3 - h ** 3) <= 1e-15


def test_p_converges_at_second_order():
    def err(n):
        x = I.grid_coords(n)
        X1, X2, X3 = np.meshgrid(x, x, x, indexing="ij")
        w = 0.1
        r2 = (X1 - 0.5) ** 2 + (X2 - 0.5) ** 2 + (X3 - 0.5) ** 2
        m = -0.3 * np.exp(-r2 / (2 * w * w))
        exact = np.stack([m * -(X - 0.5) / (w * w) for X in (X1, X2, X3)]) / (1 - m)[None]
        return np.abs(opf.gradient_p(n, m) - exact).max()
    e1, e2 = err(31), err(63)
    assert 3.5 < e1 / e2 < 4.5           # h halves: the error falls by four


def test_zero_contrast_is_the_identity():
    n = 5
    x = np.random.default_rng(1).standard_normal((3, n, n, n)) + 0j
    assert np.array_equal(opf.apply_fft_paper(n, 3.0, np.zeros((n, n, n)), x), x)
    assert np.array_equal(opf.gradient_p(n, np.zeros((n, n, n))), np.zeros((3, n, n, n)))


def _solve(n, k, apply_fn, g):
    N = 3 * n ** 3
    A = spla.LinearOperator((N, N), matvec=lambda v: apply_fn(v.reshape(3, n, n, n)).reshape(-1), dtype=complex)
    x, info = spla.gmres(A, g.reshape(-1), rtol=1e-11, atol=0.0, restart=60, maxiter=2000)
    assert info == 0
    return x.reshape(3, n, n, n)


@pytest.mark.slow
def test_paper_form_and_dyadic_form_approach_each_other():
    """Scattered fields of both forms at h = 1/8, 1/16, 1/32 compared at the
    common nodes x = i/8: the difference shrinks as h does."""
    k = 2 * math.pi * 1.0
    diffs = []
    for n in (7, 15, 31):
        x = I.grid_coords(n)
        X1, X2, X3 = np.meshgrid(x, x, x, indexing="ij")
        r2 = (X1 - 0.5) ** 2 + (X2 - 0.5) ** 2 + (X3 - 0.5) ** 2
        m = (-0.3 * np.exp(-r2 / (2 * 0.15 ** 2))).astype(complex)
        Ei = I.plane_waves(n, k, [[1.0, 0, 0]], [[0, 0, 1.0]])[0]
        Ed = _solve(n, k, lambda v: oop.apply_fft(n, k, m, v), oop.rhs_from_incident(n, k, m, Ei))
        sym = opf.paper_symbol(n, k)
        Ep = _solve(n, k, lambda v: opf.apply_fft_paper(n, k, m, v, sym),
                    opf.rhs_from_incident_paper(n, k, m, Ei, sym))
        step = (n + 1) // 8
        sl = slice(step - 1, None, step)
        d = Ed[:, sl, sl, sl] - Ep[:, sl, sl, sl]
        diffs.append(np.linalg.norm(d) / np.linalg.norm(Ed[:, sl, sl, sl]))
    print("relative difference of the two forms at x = i/8:", diffs)
    assert diffs[1] < 0.75 * diffs[0] and diffs[2] < 0.75 * diffs[1]
