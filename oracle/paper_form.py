"""The paper's own form of the discrete scattered-field equation (oracle, FP64).
TEST INFRASTRUCTURE ONLY.

Paper: Section 2, the integral form of the scattered-field equation with
p^d = (1/(1-m)) dm/dx_d and G^d = dG/dx_d, written as three scalar
convolutions with G of m E^d plus the convolutions with G^d of the scalar
p.E, and the discrete equations (the d-th component)

  E^d_i + k^2 sum_j G_ij m_j E^d_j + sum_j G^d_ij (p^1_j E^1_j + p^2_j E^2_j + p^3_j E^3_j) = g^d_i

with off-diagonal weights G_ij = h^3 G(ih - jh), G^d_ij = h^3 dG/dx_d(ih - jh).

Readings (the paper leaves these open):
  * self weights: the near-diagonal correction the paper cites is not given.
    As for the dyadic form, the self weight of G is its integral over the
    ball of volume h^3, int_ball G = e^{ika}(1/k^2 - i a/k) - 1/k^2 with
    a = h (3/(4 pi))^(1/3); that of G^d is 0 (an odd kernel's principal
    value).
  * p: not given on the grid.  p^d_j = (m_{j+e_d} - m_{j-e_d}) / (2h) / (1 - m_j),
    central differences with m = 0 outside the grid (m is supported inside
    the cube).

Functions
  gradient_p              : p on the grid (reading above).
  dG                      : the closed form of dG/dx_d.
  ball_integral_G         : the self weight of G.
  paper_weights           : (G, G^1, G^2, G^3) weights for r in [-(n-1), n-1]^3.
  apply_dense_paper       : the definition, a literal double sum (small n).
  apply_fft_paper         : zero-padded FFT convolution (four forward, three
                            inverse transforms, the 3x4 symbol multiply).
  rhs_from_incident_paper : g = E^i - A E^i.

Pins (tests/test_oracle_paper_form.py): the FFT apply equals the double sum
(brute force); dG equals a finite difference of G; the self weight equals a
quadrature of G over the ball; p converges at second order to the analytic
gradient of a Gaussian medium; m = 0 gives A x = x; the solutions of this
form and of the dyadic form approach each other as the grid is refined.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.fft

from .kernel import grid_spacing


def gradient_p(n: int, m: np.ndarray) -> np.ndarray:
    """p^d = (dm/dx_d) / (1 - m) on the grid, shape (3, n, n, n)."""
    h = grid_spacing(n)
    m = np.asarray(m, dtype=np.complex128)
    mp = np.zeros((n + 2, n + 2, n + 2), dtype=np.complex128)
    mp[1:-1, 1:-1, 1:-1] = m
    p = np.empty((3, n, n, n), dtype=np.complex128)
    c = slice(1, n + 1)
    p[0] = (mp[2:, c, c] - mp[:-2, c, c]) / (2 * h)
    p[1] = (mp[c, 2:, c] - mp[c, :-2, c]) / (2 * h)
    p[2] = (mp[c, c, 2:] - mp[c, c, :-2]) / (2 * h)
    return p / (1.0 - m)[None]


def dG(x: np.ndarray, k: float) -> np.ndarray:
    """grad G at points x (..., 3), x != 0: G(R) (ik - 1/R) x / R, shape (..., 3)."""
    x = np.asarray(x, dtype=np.float64)
    R = np.sqrt(np.sum(x * x, axis=-1))
    G = np.exp(1j * k * R) / (4.0 * math.pi * R)
    return (G * (1j * k - 1.0 / R) / R)[..., None] * x


def ball_integral_G(k: float, h: float) -> complex:
    """int of G over the ball of volume h^3 about 0: e^{ika}(1/k^2 - i a/k) - 1/k^2."""
    a = h * (3.0 / (4.0 * math.pi)) ** (1.0 / 3.0)
    return complex(np.exp(1j * k * a) * (1.0 / k ** 2 - 1j * a / k) - 1.0 / k ** 2)


def paper_weights(n: int, k: float) -> np.ndarray:
    """Weights (G, G^1, G^2, G^3) for offsets r in [-(n-1), n-1]^3, shape (4, 2n-1, 2n-1, 2n-1)."""
    h = grid_spacing(n)
    s = np.arange(-(n - 1), n, dtype=np.float64)
    r = np.stack(np.meshgrid(s, s, s, indexing="ij"), axis=-1)
    x = h * r
    R = np.sqrt(np.sum(x * x, axis=-1))
    zero = R == 0.0
    xs = np.where(zero[..., None], 1.0, x)
    Rs = np.where(zero, 1.0, R)
    out = np.empty((4,) + R.shape, dtype=np.complex128)
    out[0] = h ** 3 * np.exp(1j * k * Rs) / (4.0 * math.pi * Rs)
    out[1:] = h ** 3 * np.moveaxis(dG(xs, k), -1, 0)
    c = n - 1
    out[0, c, c, c] = ball_integral_G(k, h)
    out[1:, c, c, c] = 0.0
    return out


def apply_dense_paper(n: int, k: float, m: np.ndarray, x: np.ndarray) -> np.ndarray:
    """The definition: E^d_i + k^2 sum_j G_ij m_j E^d_j + sum_j G^d_ij (p.E)_j, literal sums."""
    W = paper_weights(n, k)
    p = gradient_p(n, m)
    m = np.asarray(m, dtype=np.complex128)
    x = np.asarray(x, dtype=np.complex128).reshape(3, n, n, n)
    u = m[None] * x
    w = np.sum(p * x, axis=0)
    y = x.copy()
    for i1 in range(n):
        for i2 in range(n):
            for i3 in range(n):
                # offsets i - j for all j: index (i - j) + n - 1
                sl = (slice(i1 + n - 1, i1 - 1 if i1 > 0 else None, -1),
                      slice(i2 + n - 1, i2 - 1 if i2 > 0 else None, -1),
                      slice(i3 + n - 1, i3 - 1 if i3 > 0 else None, -1))
                Gij = W[0][sl]
                for d in range(3):
                    y[d, i1, i2, i3] += k * k * np.sum(Gij * u[d]) + np.sum(W[1 + d][sl] * w)
    return y


def paper_symbol(n: int, k: float) -> np.ndarray:
    """Unnormalised FFT of the circulant embedding of (k^2 G, G^1, G^2, G^3), shape (4, P, P, P), P = 2n."""
    P = 2 * n
    W = paper_weights(n, k)
    W[0] *= k * k
    emb = np.zeros((4, P, P, P), dtype=np.complex128)
    s = np.arange(-(n - 1), n) % P
    emb[:, s[:, None, None], s[None, :, None], s[None, None, :]] = W
    return scipy.fft.fftn(emb, axes=(-3, -2, -1))


def apply_fft_paper(n: int, k: float, m: np.ndarray, x: np.ndarray, sym=None) -> np.ndarray:
    """A x by zero-padded FFT convolution: transforms of m E^1..3 and p.E, the 3x4 multiply, inverse."""
    P = 2 * n
    if sym is None:
        sym = paper_symbol(n, k)
    p = gradient_p(n, m)
    mm = np.asarray(m, dtype=np.complex128)
    xs = np.asarray(x, dtype=np.complex128)
    lead = xs.shape[:-4]
    xs = xs.reshape((-1, 3, n, n, n))
    out = np.empty_like(xs)
    for r in range(xs.shape[0]):
        u = np.zeros((4, P, P, P), dtype=np.complex128)
        u[:3, :n, :n, :n] = mm[None] * xs[r]
        u[3, :n, :n, :n] = np.sum(p * xs[r], axis=0)
        uh = scipy.fft.fftn(u, axes=(-3, -2, -1))
        vh = sym[0][None] * uh[:3] + sym[1:] * uh[3][None]
        v = scipy.fft.ifftn(vh, axes=(-3, -2, -1))
        out[r] = xs[r] + v[:, :n, :n, :n]
    return out.reshape(lead + (3, n, n, n))


def rhs_from_incident_paper(n: int, k: float, m: np.ndarray, Ei: np.ndarray, sym=None) -> np.ndarray:
    """g = E^i - A E^i, the right-hand side of the scattered-field equation in this form."""
    Ei = np.asarray(Ei, dtype=np.complex128)
    return Ei - apply_fft_paper(n, k, m, Ei, sym)
