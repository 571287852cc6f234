"""Seeded synthetic inputs: media, incident plane waves and random fields.

This module is shared by the GPU path's tests and benchmark and by the CPU
oracle's tests.  It holds no arithmetic of the method itself: it only draws
the contrast m(x) on the grid, incident plane waves E^i(x) = p e^{ik d.x}
and random vectors, all in complex128, from ``numpy.random.Generator(PCG64)``.

The grid follows the Nystrom discretisation of Section 2: n points per
dimension on the unit cube, spacing h = 1/(n+1), node i at x = h*i with
i in {1..n}^3.  Arrays are C-ordered ``[i1, i2, i3]`` (i3 fastest); fields
are ``[rhs, component, i1, i2, i3]``.

The paper's own test media (a Gaussian lens, a cube obstacle and a
perturbed cube, Section 4) are described by name only; smooth seeded
Gaussian media of the same kind stand in for them, and ``medium_lens``,
``medium_cube`` and ``medium_perturbed_cube`` are stated analogues of the
three named media (the shapes and contrasts are this module's choice), with
the paper's incident field E^i = (0, 0, e^{i k x_1}) (``paper_incident``).

The 2-D variant uses the n x n grid of the unit square, fields
``[rhs, component(2), i1, i2]``, the analogues ``medium2_lens``,
``medium2_square`` and ``medium2_perturbed_square`` of the paper's 2-D
examples and its incident field E^i = (0, e^{i k x_1}) (``paper_incident2``).
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def wavenumber_for(n: int, points_per_wavelength: float = 8.0) -> float:
    """k such that the unit cube spans n/ppw wavelengths (k = 2 pi n / 8)."""
    return 2.0 * math.pi * n / points_per_wavelength


def grid_coords(n: int) -> np.ndarray:
    """Node coordinates x = h*i, i = 1..n, h = 1/(n+1); shape (n,)."""
    h = 1.0 / (n + 1)
    return h * np.arange(1, n + 1, dtype=np.float64)


def _grid_mesh(n: int):
    c = grid_coords(n)
    return np.meshgrid(c, c, c, indexing="ij")


def medium_single_bump(n: int, seed: int = 0, amplitude: float = -0.2,
                       width: float = 0.15) -> np.ndarray:
    """m(x) = amplitude * exp(-|x-c|^2 / (2 width^2)), c ~ U[0.3, 0.7]^3."""
    g = _rng(seed)
    c = g.uniform(0.3, 0.7, size=3)
    x1, x2, x3 = _grid_mesh(n)
    r2 = (x1 - c[0]) ** 2 + (x2 - c[1]) ** 2 + (x3 - c[2]) ** 2
    return (amplitude * np.exp(-r2 / (2.0 * width * width))).astype(np.complex128)


def medium_lens(n: int, amplitude: float = -0.5, width: float = 0.15) -> np.ndarray:
    """Analogue of the paper's Gaussian lens: one centred Gaussian,
    m(x) = amplitude * exp(-|x - (1/2, 1/2, 1/2)|^2 / (2 width^2))
    (relative permittivity 1 - m = 1.5 at the centre)."""
    x1, x2, x3 = _grid_mesh(n)
    r2 = (x1 - 0.5) ** 2 + (x2 - 0.5) ** 2 + (x3 - 0.5) ** 2
    return (amplitude * np.exp(-r2 / (2.0 * width * width))).astype(np.complex128)


def medium_cube(n: int, amplitude: float = -0.5, side: float = 0.3, edge: float = 0.02) -> np.ndarray:
    """Analogue of the paper's cube obstacle with a smooth boundary:
    m(x) = amplitude * prod_d s(x_d), s(t) = (1 - tanh((|t - 1/2| - side/2) / edge)) / 2,
    a centred cube of the given side whose faces blur over about `edge`."""
    x1, x2, x3 = _grid_mesh(n)

    def step(t):
        return 0.5 * (1.0 - np.tanh((np.abs(t - 0.5) - side / 2) / edge))

    return (amplitude * step(x1) * step(x2) * step(x3)).astype(np.complex128)


def medium_perturbed_cube(n: int, seed: int = 0, amplitude: float = -0.5, side: float = 0.3,
                          perturbation: float = 0.2) -> np.ndarray:
    """Analogue of the paper's randomly perturbed cube obstacle: ``medium_cube``
    multiplied pointwise by 1 + perturbation * u, u ~ U[-1, 1] per grid point
    (seeded)."""
    g = _rng(seed)
    u = g.uniform(-1.0, 1.0, size=(n, n, n))
    return (medium_cube(n, amplitude, side) * (1.0 + perturbation * u)).astype(np.complex128)


PAPER_MEDIA = {"lens": medium_lens, "cube": medium_cube, "perturbed cube": medium_perturbed_cube}


def paper_wavenumber(n: int) -> float:
    """Six points per wavelength, as in the paper's tables: k = 2 pi (n + 1) / 6."""
    return 2.0 * math.pi * (n + 1) / 6.0


def medium_bumps(n: int, seed: int = 1, nbumps: int = 6, amp: float = 0.3,
                 wmin: float = 0.08, wmax: float = 0.15,
                 cmin: float = 0.2, cmax: float = 0.8,
                 min_one_minus_m: float = 0.5) -> np.ndarray:
    """Sum of ``nbumps`` seeded Gaussian bumps.

    amplitude ~ U[-amp, amp], width ~ U[wmin, wmax], centre ~ U[cmin, cmax]^3.
    A draw with min(1 - Re m) < ``min_one_minus_m`` is rejected and redrawn
    from the next sub-seed, deterministically.
    """
    x1, x2, x3 = _grid_mesh(n)
    for sub in range(1000):
        g = _rng(seed * 1000 + sub)
        m = np.zeros((n, n, n), dtype=np.float64)
        for _ in range(nbumps):
            a = g.uniform(-amp, amp)
            w = g.uniform(wmin, wmax)
            c = g.uniform(cmin, cmax, size=3)
            r2 = (x1 - c[0]) ** 2 + (x2 - c[1]) ** 2 + (x3 - c[2]) ** 2
            m += a * np.exp(-r2 / (2.0 * w * w))
        if np.min(1.0 - m) >= min_one_minus_m:
            return m.astype(np.complex128)
    raise RuntimeError("medium_bumps: no admissible draw")


def medium_random_complex(n: int, seed: int, scale: float = 0.3) -> np.ndarray:
    """Unstructured complex contrast, for operator parity tests only."""
    g = _rng(seed)
    return scale * (g.standard_normal((n, n, n)) + 1j * g.standard_normal((n, n, n)))


def random_field(nrhs: int, n: int, seed: int) -> np.ndarray:
    """Complex standard-normal field, shape (nrhs, 3, n, n, n)."""
    g = _rng(seed)
    shp = (nrhs, 3, n, n, n)
    return g.standard_normal(shp) + 1j * g.standard_normal(shp)


def polarisation_basis(d: np.ndarray):
    """Two unit vectors p1, p2 with p1 . d = p2 . d = 0 and p2 = d x p1.

    p1 is e3 projected off d (e1 when d is within ~25 degrees of e3).
    """
    d = np.asarray(d, dtype=np.float64)
    d = d / np.linalg.norm(d)
    e = np.array([0.0, 0.0, 1.0]) if abs(d[2]) <= 0.9 else np.array([1.0, 0.0, 0.0])
    p1 = e - np.dot(e, d) * d
    p1 /= np.linalg.norm(p1)
    p2 = np.cross(d, p1)
    return p1, p2


def random_direction_and_polarisation(seed: int):
    """d uniform on the sphere; p = cos(t) p1 + sin(t) p2, t ~ U[0, 2 pi)."""
    g = _rng(seed)
    d = g.standard_normal(3)
    d /= np.linalg.norm(d)
    t = g.uniform(0.0, 2.0 * math.pi)
    p1, p2 = polarisation_basis(d)
    return d, math.cos(t) * p1 + math.sin(t) * p2


def fibonacci_directions(count: int) -> np.ndarray:
    """Directions z_j = 1 - (2j+1)/count, phi_j = j pi (3 - sqrt 5); (count, 3)."""
    j = np.arange(count, dtype=np.float64)
    z = 1.0 - (2.0 * j + 1.0) / count
    phi = j * math.pi * (3.0 - math.sqrt(5.0))
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def fibonacci_incident_set(count: int):
    """(directions, polarisations): each direction with its two polarisations."""
    dirs, pols = [], []
    for d in fibonacci_directions(count):
        p1, p2 = polarisation_basis(d)
        dirs += [d, d]
        pols += [p1, p2]
    return np.array(dirs), np.array(pols)


def plane_waves(n: int, k: float, dirs, pols) -> np.ndarray:
    """E^i_c(x) = p_c exp(i k d.x) on the grid; shape (len(dirs), 3, n, n, n)."""
    x1, x2, x3 = _grid_mesh(n)
    dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
    pols = np.atleast_2d(np.asarray(pols, dtype=np.float64))
    out = np.empty((len(dirs), 3, n, n, n), dtype=np.complex128)
    for r, (d, p) in enumerate(zip(dirs, pols)):
        phase = np.exp(1j * k * (d[0] * x1 + d[1] * x2 + d[2] * x3))
        for c in range(3):
            out[r, c] = p[c] * phase
    return out


def paper_incident(n: int, k: float) -> np.ndarray:
    """The incident field of the paper's 3-D examples, E^i = (0, 0, e^{i k x_1});
    shape (1, 3, n, n, n)."""
    return plane_waves(n, k, [[1.0, 0.0, 0.0]], [[0.0, 0.0, 1.0]])


# --- the 2-D variant: n x n grid of the unit square, fields [rhs, component(2), i1, i2] ---

def _grid_mesh2(n: int):
    x = grid_coords(n)
    return np.meshgrid(x, x, indexing="ij")


def medium2_lens(n: int, amplitude: float = -0.5, width: float = 0.15) -> np.ndarray:
    """2-D analogue of the paper's converging Gaussian lens (Section 4, 2-D
    examples): m(x) = amplitude * exp(-|x - (1/2, 1/2)|^2 / (2 width^2))."""
    x1, x2 = _grid_mesh2(n)
    r2 = (x1 - 0.5) ** 2 + (x2 - 0.5) ** 2
    return (amplitude * np.exp(-r2 / (2.0 * width * width))).astype(np.complex128)


def medium2_square(n: int, amplitude: float = -0.5, side: float = 0.3, edge: float = 0.02) -> np.ndarray:
    """2-D analogue of the paper's square obstacle with a smooth boundary:
    amplitude * s(x_1) s(x_2), s(t) = (1 - tanh((|t - 1/2| - side/2) / edge)) / 2."""
    x1, x2 = _grid_mesh2(n)

    def step(t):
        return 0.5 * (1.0 - np.tanh((np.abs(t - 0.5) - side / 2) / edge))

    return (amplitude * step(x1) * step(x2)).astype(np.complex128)


def medium2_perturbed_square(n: int, seed: int = 0, amplitude: float = -0.5, side: float = 0.3,
                             perturbation: float = 0.2) -> np.ndarray:
    """2-D analogue of the paper's random perturbation of the square obstacle:
    ``medium2_square`` times 1 + perturbation * u, u ~ U[-1, 1] per point (seeded)."""
    u = _rng(seed).uniform(-1.0, 1.0, size=(n, n))
    return (medium2_square(n, amplitude, side) * (1.0 + perturbation * u)).astype(np.complex128)


PAPER_MEDIA_2D = {"lens": medium2_lens, "square": medium2_square, "perturbed square": medium2_perturbed_square}


def medium2_random_complex(n: int, seed: int, scale: float = 0.3) -> np.ndarray:
    """Unstructured complex 2-D contrast, for operator parity tests only."""
    g = _rng(seed)
    return scale * (g.standard_normal((n, n)) + 1j * g.standard_normal((n, n)))


def random_field2(nrhs: int, n: int, seed: int) -> np.ndarray:
    """Complex standard-normal 2-D field, shape (nrhs, 2, n, n)."""
    g = _rng(seed)
    shp = (nrhs, 2, n, n)
    return g.standard_normal(shp) + 1j * g.standard_normal(shp)


def plane_waves2(n: int, k: float, dirs, pols) -> np.ndarray:
    """E^i_c(x) = p_c exp(i k d.x) on the 2-D grid; shape (len(dirs), 2, n, n)."""
    x1, x2 = _grid_mesh2(n)
    dirs = np.atleast_2d(np.asarray(dirs, dtype=np.float64))
    pols = np.atleast_2d(np.asarray(pols, dtype=np.float64))
    out = np.empty((len(dirs), 2, n, n), dtype=np.complex128)
    for r, (d, p) in enumerate(zip(dirs, pols)):
        phase = np.exp(1j * k * (d[0] * x1 + d[1] * x2))
        for c in range(2):
            out[r, c] = p[c] * phase
    return out


def circle_incident_set2(count: int):
    """``count`` directions evenly spaced on the circle, each with its in-plane
    polarisation p = (-d_2, d_1): (directions, polarisations)."""
    t = 2.0 * math.pi * np.arange(count) / count
    d = np.stack([np.cos(t), np.sin(t)], axis=1)
    return d, np.stack([-d[:, 1], d[:, 0]], axis=1)


def paper_incident2(n: int, k: float) -> np.ndarray:
    """The incident field of the paper's 2-D examples, E^i = (0, e^{i k x_1});
    shape (1, 2, n, n)."""
    return plane_waves2(n, k, [[1.0, 0.0]], [[0.0, 1.0]])
