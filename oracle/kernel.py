"""Grid and dyadic Green's tensor (oracle, FP64).  TEST INFRASTRUCTURE ONLY.

Paper: Section 2 (Problem formulation).  The Helmholtz kernel is
G(x) = exp(ik|x|) / (4 pi |x|) (after Eq. (3)); the grid is the uniform
Cartesian grid of the Nystrom discretisation, h = 1/(n+1), nodes x_i = i h
(before Eq. (5)); off-diagonal matrix entries are h^3 times kernel samples
(after Eq. (5)).

Reading taken here (dyadic form): the operator is written as
E + K * (m E) with K = (k^2 I + grad grad) G, the dyadic Green's tensor.
In the continuum this is the same equation as Eq. (4): the divergence of
(1-m)E vanishes, so grad G * (div(m E)) equals the paper's
grad G * (p . E) with p = grad m / (1 - m).  Away from the origin

  K(x) = G(R) [ (k^2 + ik/R - 1/R^2) I + (-k^2 - 3ik/R + 3/R^2) xhat xhat^T ],

and the Nystrom weight is h^3 K(h r) for r != 0.

Self term (the paper uses a fourth-order correction whose weights it does not
give): the cell is replaced by the ball of equal volume, radius
a = h (3/(4 pi))^(1/3), and K(0) is the principal-value integral of the
tensor over that ball plus the -1/3 depolarisation term:

  K(0) = { (2/3) [ (1 - ika) e^{ika} - 1 ] - 1/3 } I.

Pins (tests/test_oracle_kernel.py): closed form against mpmath finite
differences of G; ball integral against mpmath quadrature; symmetry,
evenness and cubic covariance; the Helmholtz equation away from 0.  With the
operator (tests/test_oracle_physics.py): the total field inside a small
homogeneous sphere is the static 3 E0 / (eps + 2), eps = 1 - m, to first order
in h, which fixes the self term's -1/3 depolarisation.
"""
from __future__ import annotations

import math

import numpy as np


def grid_spacing(n: int) -> float:
    """h = 1/(n+1) (Section 2, before Eq. (5))."""
    return 1.0 / (n + 1)


def helmholtz_G(R, k):
    """G(R) = exp(ikR)/(4 pi R) (Section 2, after Eq. (3))."""
    R = np.asarray(R, dtype=np.float64)
    return np.exp(1j * k * R) / (4.0 * math.pi * R)


def self_term(k: float, h: float) -> complex:
    """Scalar s with K(0) = s I: equal-volume-ball principal value + depolarisation."""
    a = h * (3.0 / (4.0 * math.pi)) ** (1.0 / 3.0)
    ball = (1.0 - 1j * k * a) * np.exp(1j * k * a) - 1.0   # k^2 * integral of G over the ball
    return complex((2.0 / 3.0) * ball - 1.0 / 3.0)


def dyadic_tensor(r, k: float, h: float) -> np.ndarray:
    """Nystrom weights K(r), r integer offsets of shape (..., 3) -> (..., 3, 3) complex.

    r != 0: h^3 (k^2 I + grad grad) G at x = h r.  r == 0: the self term.
    """
    r = np.asarray(r, dtype=np.float64)
    shp = r.shape[:-1]
    x = h * r
    R = np.sqrt(np.sum(x * x, axis=-1))
    zero = R == 0.0
    Rs = np.where(zero, 1.0, R)
    G = np.exp(1j * k * Rs) / (4.0 * math.pi * Rs)
    c_iso = G * (k * k + 1j * k / Rs - 1.0 / Rs ** 2)
    c_rad = G * (-k * k - 3j * k / Rs + 3.0 / Rs ** 2)
    xh = x / Rs[..., None]
    eye = np.eye(3)
    out = h ** 3 * (c_iso[..., None, None] * eye
                    + c_rad[..., None, None] * xh[..., :, None] * xh[..., None, :])
    if np.any(zero):
        out[zero] = self_term(k, h) * eye
    return out.reshape(shp + (3, 3))


def kernel_table(n: int, k: float) -> np.ndarray:
    """K(r) for every r in [-(n-1), n-1]^3, shape (2n-1, 2n-1, 2n-1, 3, 3).

    Index [r1 + n-1, r2 + n-1, r3 + n-1].
    """
    h = grid_spacing(n)
    s = np.arange(-(n - 1), n, dtype=np.float64)
    r = np.stack(np.meshgrid(s, s, s, indexing="ij"), axis=-1)
    return dyadic_tensor(r, k, h)
