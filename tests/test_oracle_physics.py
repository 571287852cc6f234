"""Physical pins of the oracle's discretisation (CPU).

The closed forms of the static limit fix the total field inside a homogeneous
scatterer that is small against the wavelength: a uniform incident field E0
gives the uniform interior field 3 E0 / (eps + 2) in a sphere and, for an
in-plane field, 2 E0 / (eps + 1) in a circular cylinder, with eps = 1 - m the
relative permittivity (the paper writes p = grad m / (1 - m), so 1 - m is the
permittivity).  The discrete equations reach these values only if the self
term, the depolarisation and the gradient term are right: dropping the -1/3 of
the 3-D self term gives about 1.0 instead of 0.857 at m = -0.5, a flipped
sign 1.2, and in 2-D a dropped or sign-flipped p.E term misses by 25 %.

The 3-D dyadic form converges to the closed form at first order in h (the
staircase sphere).  The 2-D paper form keeps an error of about 1 % as h -> 0:
its central difference of m over a jump, divided by 1 - m, integrates to
0.417 where the jump of log(1 - m) is 0.405 (m = -0.5), so the bound here is
2 %.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as sla

from oracle import operator as op
from oracle import two_d as T
from oracle.kernel import grid_spacing

K_STATIC = 0.05   # k |x| < 0.05 over the unit cube: static up to ~1e-3


def _solve(N, matvec, b):
    A = sla.LinearOperator((N, N), matvec=matvec, dtype=np.complex128)
    x, info = sla.gmres(A, b, rtol=1e-10, restart=60, maxiter=400)
    assert info == 0
    return x


def sphere_interior_field(n: int, mval: float, R: float = 0.3):
    """Mean of E_z / E0_z over points deeper than 1.5 h inside a ball of radius R
    (total field of A E = E^i, z-polarised field propagating along x_1), and the
    largest cross-polarised |E_x| there."""
    k = K_STATIC
    h = grid_spacing(n)
    x = (np.arange(n) + 1) * h
    X1, X2, X3 = np.meshgrid(x, x, x, indexing="ij")
    r = np.sqrt((X1 - .5) ** 2 + (X2 - .5) ** 2 + (X3 - .5) ** 2)
    m = np.where(r < R, mval, 0.0).astype(np.complex128)
    Kh = op.kernel_symbol(n, k)
    Ei = np.zeros((3, n, n, n), np.complex128)
    Ei[2] = np.exp(1j * k * X1)
    E = _solve(3 * n ** 3, lambda v: op.apply_fft(n, k, m, v.reshape(3, n, n, n), Kh).reshape(-1),
               Ei.reshape(-1)).reshape(3, n, n, n)
    deep = r < R - 1.5 * h
    return float((E[2] / Ei[2])[deep].real.mean()), float(np.abs(E[0][deep]).max())


def cylinder_interior_field(n: int, mval: float, R: float = 0.3):
    """2-D: mean of E^2 / E0^2 over points deeper than 2.5 h inside a disc of
    radius R (field polarised along x_2, propagating along x_1)."""
    k = K_STATIC
    h = T.grid_spacing(n)
    x = (np.arange(n) + 1) * h
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    r = np.sqrt((X1 - .5) ** 2 + (X2 - .5) ** 2)
    m = np.where(r < R, mval, 0.0).astype(np.complex128)
    sym = T.symbol2(n, k)
    Ei = np.zeros((2, n, n), np.complex128)
    Ei[1] = np.exp(1j * k * X1)
    E = _solve(2 * n * n, lambda v: T.apply_fft2(n, k, m, v.reshape(2, n, n), sym).reshape(-1),
               Ei.reshape(-1)).reshape(2, n, n)
    deep = r < R - 2.5 * h
    return float((E[1] / Ei[1])[deep].real.mean()), float(np.abs(E[0][deep]).max())


@pytest.mark.parametrize("mval", [-0.5, 0.4])
def test_sphere_static_limit(mval):
    """Self term and dyadic kernel: 3 / (eps + 2) inside a small sphere, n = 16."""
    mean, cross = sphere_interior_field(16, mval)
    exact = 3.0 / (3.0 - mval)
    assert abs(mean / exact - 1) < 0.01, (mean, exact)
    assert cross < 0.02


def test_sphere_static_limit_converges():
    """A strong contrast (eps = 3): the error falls with h (first order)."""
    exact = 3.0 / 5.0
    e12 = abs(sphere_interior_field(12, -2.0)[0] / exact - 1)
    e24 = abs(sphere_interior_field(24, -2.0)[0] / exact - 1)
    assert e24 < 0.02 and e24 < 0.6 * e12, (e12, e24)


@pytest.mark.parametrize("mval", [-0.5, 0.4])
def test_cylinder_static_limit(mval):
    """2-D paper form (k^2 G and the p.E gradient term): 2 / (eps + 1) inside a
    small cylinder, n = 80, within the 2 % that its jump discretisation leaves."""
    mean, cross = cylinder_interior_field(80, mval)
    exact = 2.0 / (2.0 - mval)
    assert abs(mean / exact - 1) < 0.02, (mean, exact)
    assert cross < 0.03
