"""Pins of the oracle's dyadic kernel against mathematics independent of its code.

* closed form of (k^2 I + grad grad) G against mpmath derivatives of
  G(x) = exp(ik|x|)/(4 pi |x|) (Section 2, after Eq. (3));
* divergence-free columns away from the origin (div K = k^2 grad G + grad Delta G = 0);
* self term against a numerical principal-value quadrature over the ball;
* symmetry, evenness and covariance under the cubic group.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import kernel as K


def _G_mp(k):
    def G(x1, x2, x3):
        R = mp.sqrt(x1 ** 2 + x2 ** 2 + x3 ** 2)
        return mp.exp(1j * k * R) / (4 * mp.pi * R)
    return G


@pytest.mark.parametrize("n,seed", [(8, 0), (16, 1), (40, 2)])
def test_closed_form_matches_mpmath_hessian(n, seed):
    mp.mp.dps = 30
    k = 2 * math.pi * n / 8
    h = K.grid_spacing(n)
    G = _G_mp(k)
    rng = np.random.default_rng(seed)
    for _ in range(6):
        r = rng.integers(-(n - 1), n, size=3)
        if not r.any():
            continue
        x = [mp.mpf(h * float(v)) for v in r]
        H = np.zeros((3, 3), complex)
        for a in range(3):
            for b in range(3):
                o = [0, 0, 0]
                o[a] += 1
                o[b] += 1
                H[a, b] = complex(mp.diff(G, x, tuple(o)))
        ref = h ** 3 * (k * k * complex(G(*x)) * np.eye(3) + H)
        got = K.dyadic_tensor(r, k, h)
        assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_columns_divergence_free():
    """div K = k^2 grad G + grad(Delta G) = 0 off the origin (central differences)."""
    n = 16
    k = 2 * math.pi * 2
    h = K.grid_spacing(n)
    r0 = np.array([3.0, -2.0, 5.0])
    dr = 1e-4
    div = np.zeros(3, complex)
    for a in range(3):
        e = np.zeros(3)
        e[a] = dr
        dK = (K.dyadic_tensor(r0 + e, k, h) - K.dyadic_tensor(r0 - e, k, h)) / (2 * dr * h)
        div += dK[a, :]
    scale = np.abs(K.dyadic_tensor(r0, k, h)).max() / (h * np.linalg.norm(r0))
    assert np.abs(div).max() <= 1e-6 * scale
    # and a non-zero control: the gradient of one column is not small
    assert np.abs(dK).max() > 1e-2 * scale


def _pv_ball_quadrature(k, a, nr=80, nt=24, nph=24, eps=1e-3):
    """Principal-value integral of (k^2 + grad grad)G over |x| < a (shell eps < R < a)."""
    R, wR = np.polynomial.legendre.leggauss(nr)
    R = eps * a + (a - eps * a) * (R + 1) / 2
    wR = wR * (a - eps * a) / 2
    ct, wt = np.polynomial.legendre.leggauss(nt)
    ph = 2 * math.pi * np.arange(nph) / nph
    wph = 2 * math.pi / nph
    tot = np.zeros((3, 3), complex)
    for Ri, wi in zip(R, wR):
        for c, wc in zip(ct, wt):
            s = math.sqrt(1 - c * c)
            for p in ph:
                xh = np.array([s * math.cos(p), s * math.sin(p), c])
                G = np.exp(1j * k * Ri) / (4 * math.pi * Ri)
                T = G * ((k * k + 1j * k / Ri - 1 / Ri ** 2) * np.eye(3)
                         + (-k * k - 3j * k / Ri + 3 / Ri ** 2) * np.outer(xh, xh))
                tot += wi * wc * wph * Ri * Ri * T
    # the inner ball eps*a contributes k^2 * int G (isotropic part) -> O(eps^2): added exactly
    ri = eps * a
    inner = ((1 - 1j * k * ri) * np.exp(1j * k * ri) - 1) * (2.0 / 3.0)
    return tot + inner * np.eye(3)


@pytest.mark.parametrize("n", [16, 64])
def test_self_term_matches_ball_quadrature(n):
    k = 2 * math.pi * n / 8
    h = K.grid_spacing(n)
    a = h * (3 / (4 * math.pi)) ** (1 / 3)
    pv = _pv_ball_quadrature(k, a)
    expect = pv - np.eye(3) / 3.0           # delta part of grad grad (1/4piR): -I/3
    got = K.dyadic_tensor(np.zeros(3), k, h)
    assert np.abs(got - expect).max() <= 1e-10
    # equal-volume ball: 4/3 pi a^3 = h^3
    assert abs(4 / 3 * math.pi * a ** 3 - h ** 3) < 1e-18


def test_symmetry_and_cubic_covariance():
    n = 12
    k = 2 * math.pi * 1.5
    h = K.grid_spacing(n)
    T = K.kernel_table(n, k)
    c = n - 1
    # K(r) = K(r)^T = K(-r)
    assert np.allclose(T, np.swapaxes(T, -1, -2), rtol=0, atol=1e-15 * np.abs(T).max())
    assert np.allclose(T, T[::-1, ::-1, ::-1], rtol=0, atol=1e-15 * np.abs(T).max())
    # reflection r_d -> -r_d flips the sign of entries (a, b) with exactly one index = d
    for d in range(3):
        R = np.eye(3)
        R[d, d] = -1
        Tr = np.flip(T, axis=d)
        assert np.allclose(Tr, R @ T @ R, rtol=0, atol=1e-15 * np.abs(T).max())
    # permutation covariance K(P r) = P K(r) P^T
    rng = np.random.default_rng(0)
    for perm in [(1, 0, 2), (2, 0, 1), (0, 2, 1)]:
        Pm = np.eye(3)[list(perm)]
        for _ in range(20):
            r = rng.integers(-c, c + 1, size=3)
            lhs = K.dyadic_tensor(Pm @ r, k, h)
            rhs = Pm @ K.dyadic_tensor(r, k, h) @ Pm.T
            assert np.abs(lhs - rhs).max() <= 1e-14 * np.abs(rhs).max()
