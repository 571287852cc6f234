"""Pins of the oracle's 2-D variant (Section 2 in two dimensions, Sections
3.1-3.2 stencils, Section 4 2-D examples).

Each pin checks the oracle against something other than its own formula:
the literal double sum, the known singular and far-field behaviour of the
2-D fundamental solution, finite differences, quadrature, the convergence
order of p, the Ky Fan bound of the fit, the mirror symmetry between
boundary classes, Gauss's law for the computed field, and the paper's
iteration counts.
"""
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.sparse.linalg as spla
import scipy.special

from oracle import fgmres as ofg
from oracle import sparse as osp
from oracle import two_d as o2
from paper_1804_02297_amd import inputs as I


@pytest.mark.parametrize("n", [3, 4, 5, 7])
def test_fft_apply_equals_double_sum(n):
    g = np.random.default_rng(n)
    m = 0.2 * (g.standard_normal((n, n)) + 1j * g.standard_normal((n, n)))
    x = g.standard_normal((2, n, n)) + 1j * g.standard_normal((2, n, n))
    k = 2 * math.pi * 1.3
    a = o2.apply_fft2(n, k, m, x)
    b = o2.apply_dense2(n, k, m, x)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


def test_kernel_is_the_outgoing_fundamental_solution():
    k = 9.0
    # logarithmic singularity of -Laplace^-1: G(r1) - G(r2) -> -(1/2 pi) ln(r1 / r2)
    r1, r2 = 1e-7, 2e-7
    assert abs((o2.G2(r1, k) - o2.G2(r2, k)) - (-math.log(r1 / r2) / (2 * math.pi))) < 1e-10
    # Helmholtz equation away from 0 (five-point Laplacian, step d)
    d = 1e-3
    for x0 in ([0.3, 0.1], [-0.2, 0.45]):
        x0 = np.array(x0)
        f = lambda y: o2.G2(np.linalg.norm(y), k)
        lap = sum(f(x0 + d * e) + f(x0 - d * e) - 2 * f(x0) for e in np.eye(2)) / d ** 2
        assert abs(lap + k * k * f(x0)) <= 1e-5 * abs(k * k * f(x0))
    # outgoing far field: G ~ (i/4) sqrt(2 / (pi k R)) e^{i (k R - pi/4)}
    R = 4000.0
    far = 0.25j * math.sqrt(2 / (math.pi * k * R)) * np.exp(1j * (k * R - math.pi / 4))
    assert abs(o2.G2(R, k) - far) <= 1e-4 * abs(far)


def test_gradient_of_G_matches_finite_differences():
    k = 7.0
    d = 1e-6
    for x in ([0.3, -0.2], [0.05, 0.4], [-0.6, 0.0]):
        x = np.array(x)
        num = np.array([(o2.G2(np.linalg.norm(x + d * e), k) - o2.G2(np.linalg.norm(x - d * e), k)) / (2 * d)
                        for e in np.eye(2)])
        assert np.abs(o2.dG2(x, k) - num).max() <= 1e-7 * np.abs(num).max()


@pytest.mark.parametrize("k,h", [(5.0, 0.05), (60.0, 1 / 120), (300.0, 1 / 960)])
def test_self_weight_is_the_disc_integral(k, h):
    a = h / math.sqrt(math.pi)
    # int_disc (i/4) H0(k r) dA = (i pi / 2) int_0^a r H0(k r) dr
    re = scipy.integrate.quad(lambda r: r * scipy.special.jv(0, k * r), 0, a, epsabs=0, epsrel=1e-13)[0]
    im = scipy.integrate.quad(lambda r: r * scipy.special.yv(0, k * r), 0, a, epsabs=0, epsrel=1e-12, limit=200)[0]
    ref = 0.5j * math.pi * (re + 1j * im)
    assert abs(o2.disc_integral_G2(k, h) - ref) <= 1e-10 * abs(ref)
    assert abs(math.pi * a * a - h * h) <= 1e-15


def test_p_converges_at_second_order():
    def err(n):
        x = I.grid_coords(n)
        X1, X2 = np.meshgrid(x, x, indexing="ij")
        w = 0.1
        m = -0.3 * np.exp(-((X1 - 0.5) ** 2 + (X2 - 0.5) ** 2) / (2 * w * w))
        exact = np.stack([m * -(X - 0.5) / (w * w) for X in (X1, X2)]) / (1 - m)[None]
        return np.abs(o2.gradient_p2(n, m) - exact).max()
    e1, e2 = err(63), err(127)
    assert 3.5 < e1 / e2 < 4.5


def test_zero_contrast_is_the_identity():
    n = 6
    x = np.random.default_rng(2).standard_normal((2, n, n)) + 0j
    assert np.array_equal(o2.apply_fft2(n, 3.0, np.zeros((n, n)), x), x)


def test_fit_attains_the_ky_fan_minimum():
    n, k = 12, I.paper_wavenumber(12)
    for kappa in range(9):
        alpha, beta, _ = o2.fit_class2(kappa, n, k)
        tau = o2.tau_offsets2(kappa)
        M = o2.coupling_block2(tau, o2.complement_offsets2(kappa, n), n, k)
        ev = np.linalg.eigvalsh(M @ M.conj().T)                    # ascending
        assert np.allclose(alpha.conj().T @ alpha, np.eye(2), atol=1e-12)
        assert abs(np.linalg.norm(alpha.conj().T @ M) ** 2 - ev[:2].sum()) <= 1e-9 * ev[-1]
        # the local stencil is far more local than a point evaluation
        e = np.zeros((len(alpha), 2))
        e[2 * list(map(tuple, tau)).index((0, 0)), 0] = 1
        e[2 * list(map(tuple, tau)).index((0, 0)) + 1, 1] = 1
        assert np.linalg.norm(alpha.conj().T @ M) < 0.2 * np.linalg.norm(e.T @ M)


def test_boundary_classes_are_mirror_images():
    """Reflecting x_1 -> -x_1 maps class (lo, c2) to (hi, c2): G and G^2 are
    even and G^1 odd in x_1, so the reflected alpha with its component 1 and
    the p.E column negated spans the other class's subspace."""
    n, k = 10, I.paper_wavenumber(10)
    for c2 in range(3):
        a_lo, b_lo, _ = o2.fit_class2(3 * 0 + c2, n, k)
        a_hi, b_hi, _ = o2.fit_class2(3 * 2 + c2, n, k)
        tau_lo = [tuple(t) for t in o2.tau_offsets2(c2)]
        tau_hi = [tuple(t) for t in o2.tau_offsets2(6 + c2)]
        perm = [tau_lo.index((-t[0], t[1])) for t in tau_hi]
        mapped = np.zeros_like(a_lo)
        for th, tl in enumerate(perm):
            mapped[2 * th] = -a_lo[2 * tl]
            mapped[2 * th + 1] = a_lo[2 * tl + 1]
        P1 = a_hi @ a_hi.conj().T
        P2 = mapped @ mapped.conj().T
        assert np.abs(P1 - P2).max() <= 1e-9


def _solve_total_field(n, k, m, tol=1e-11):
    Ei = I.paper_incident2(n, k)[0]
    sym = o2.symbol2(n, k)
    g = o2.rhs2(n, k, m, Ei, sym)
    N = 2 * n * n
    A = spla.LinearOperator((N, N), matvec=lambda v: o2.apply_fft2(n, k, m, v.reshape(2, n, n), sym).reshape(-1),
                            dtype=complex)
    Es, info = spla.gmres(A, g.reshape(-1), rtol=tol, atol=0.0, restart=80, maxiter=3000)
    assert info == 0
    return Ei + Es.reshape(2, n, n)


@pytest.mark.slow
def test_solution_satisfies_gauss_law():
    """div((1 - m) E) = 0 for the exact field; its central difference on the
    grid falls at second order as h halves (a sign or index error in the
    G^d p.E term leaves an O(1) divergence)."""
    k = 2 * math.pi * 2.0
    res = []
    for n in (31, 63):
        h = 1.0 / (n + 1)
        m = I.medium2_lens(n, amplitude=-0.3, width=0.12)
        E = _solve_total_field(n, k, m)
        D = (1 - m)[None] * E
        div = (D[0, 2:, 1:-1] - D[0, :-2, 1:-1]) / (2 * h) + (D[1, 1:-1, 2:] - D[1, 1:-1, :-2]) / (2 * h)
        scale = np.abs((D[1, 1:-1, 2:] - D[1, 1:-1, :-2]) / (2 * h)).max()
        res.append(np.abs(div).max() / scale)
    print("relative divergence at n = 31, 63:", res)
    assert res[0] < 0.15 and res[1] < res[0] / 3


def test_preconditioned_gmres_takes_few_iterations():
    """The paper's 2-D claim (six iterations at six points per wavelength)
    on the analogue of its square obstacle, with S^-1 Q from the class
    stencils: 4 iterations against 16 without it.  Dropping the p.E part of
    beta (a plausible assembly mistake) already costs 7."""
    n = 39
    k = I.paper_wavenumber(n)
    m = I.medium2_square(n)
    alphas, betas, _ = o2.fit_all_classes2(n, k)
    S, Q = o2.assemble2(n, m, alphas, betas)
    P = osp.Preconditioner(S, Q)
    sym = o2.symbol2(n, k)
    g = o2.rhs2(n, k, m, I.paper_incident2(n, k)[0], sym)
    x, info = ofg.fgmres(lambda v: o2.apply_fft2(n, k, m, v, sym), g, P, tol=1e-6, restart=20)
    _, info0 = ofg.fgmres(lambda v: o2.apply_fft2(n, k, m, v, sym), g, None, tol=1e-6, restart=20, maxit=400)
    print("iterations with / without the preconditioner:", info["iters"], info0["iters"])
    assert info["rel_resid"] <= 1e-6 and info["iters"] <= 5
    assert info0["iters"] > 3 * info["iters"]


def test_zero_contrast_rows():
    """m = 0: S = Q, so the preconditioner is the identity on A = I."""
    n = 8
    k = I.paper_wavenumber(n)
    alphas, betas, _ = o2.fit_all_classes2(n, k)
    S, Q = o2.assemble2(n, np.zeros((n, n)), alphas, betas)
    assert (S - Q).count_nonzero() == 0 or abs(S - Q).max() == 0
    P = osp.Preconditioner(S, Q)
    v = np.random.default_rng(0).standard_normal((2, n, n)) + 0j
    assert np.abs(P(v) - v).max() <= 1e-12
