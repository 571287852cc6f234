"""The seeded input generators for the paper's media analogues (CPU only)."""
import math

import numpy as np

from paper_1804_02297_amd import inputs as I


def test_paper_wavenumber_is_six_points_per_wavelength():
    for n in (29, 59, 119):
        k = I.paper_wavenumber(n)
        h = 1.0 / (n + 1)
        assert abs((2 * math.pi / k) / h - 6.0) < 1e-12
    # the paper's tables: k / 2 pi = 5, 10, 20 at N = 3 x 29^3, 3 x 59^3, 3 x 119^3
    assert [round(I.paper_wavenumber(n) / (2 * math.pi), 12) for n in (29, 59, 119)] == [5, 10, 20]


def test_lens_is_a_centred_symmetric_gaussian():
    n = 29
    m = I.medium_lens(n)
    assert np.abs(m.imag).max() == 0
    c = n // 2                                   # x = 1/2 on an odd grid
    assert abs(m[c, c, c] + 0.5) < 1e-15 and np.argmin(m.real) == np.ravel_multi_index((c, c, c), m.shape)
    for axis in range(3):                        # x -> 1 - x is index i -> n - 1 - i
        assert np.allclose(m, np.flip(m, axis))
    assert np.allclose(m, m.transpose(1, 0, 2)) and np.allclose(m, m.transpose(2, 1, 0))


def test_cube_has_its_value_inside_and_a_smooth_edge():
    n = 59
    m = I.medium_cube(n).real
    x = I.grid_coords(n)
    c = n // 2
    assert abs(m[c, c, c] + 0.5) < 1e-6          # deep inside: the full contrast
    assert abs(m[0, 0, 0]) < 1e-12               # far outside: none
    # along an axis through the centre the profile is monotone in |x - 1/2| and
    # half of the contrast is reached at the face |x - 1/2| = side / 2
    prof = m[:, c, c]
    d = np.abs(x - 0.5)
    order = np.argsort(d)
    assert np.all(np.diff(np.abs(prof[order])) <= 1e-15)
    step = 0.5 * (1 - np.tanh((d - 0.15) / 0.02))
    assert np.allclose(prof, -0.5 * step * step[c] * step[c])


def test_perturbed_cube_is_seeded_and_bounded():
    n = 29
    a = I.medium_perturbed_cube(n, seed=3)
    b = I.medium_perturbed_cube(n, seed=3)
    c = I.medium_perturbed_cube(n, seed=4)
    base = I.medium_cube(n)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    ratio = a.real[np.abs(base) > 1e-3] / base.real[np.abs(base) > 1e-3]
    assert ratio.min() >= 0.8 - 1e-12 and ratio.max() <= 1.2 + 1e-12 and ratio.std() > 0.05


def test_paper_incident_field():
    n, k = 9, I.paper_wavenumber(9)
    e = I.paper_incident(n, k)
    x1 = I.grid_coords(n)[:, None, None]
    assert np.array_equal(e[0, 0], np.zeros((n, n, n))) and np.array_equal(e[0, 1], np.zeros((n, n, n)))
    assert np.allclose(e[0, 2], np.broadcast_to(np.exp(1j * k * x1), (n, n, n)))


def test_two_d_generators():
    n = 9
    k = I.paper_wavenumber(n)
    Ei = I.paper_incident2(n, k)
    x = I.grid_coords(n)
    assert Ei.shape == (1, 2, n, n)
    assert np.array_equal(Ei[0, 0], np.zeros((n, n)))
    assert np.allclose(Ei[0, 1], np.exp(1j * k * x)[:, None] * np.ones(n)[None])
    d, p = I.circle_incident_set2(6)
    assert np.allclose(np.sum(d * p, axis=1), 0) and np.allclose(np.linalg.norm(p, axis=1), 1)
    assert np.array_equal(I.medium2_perturbed_square(n, 3), I.medium2_perturbed_square(n, 3))
    assert abs(I.medium2_lens(n)[n // 2, n // 2] + 0.5) < 1e-12
    assert I.random_field2(2, n, 1).shape == (2, 2, n, n)
