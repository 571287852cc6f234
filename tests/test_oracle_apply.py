"""Pins of the oracle's Nystrom apply A x = x + K * (m x) (Eq. (5), Eq. (6)).

* brute force: the literal double sum equals the zero-padded FFT apply;
* m = 0: A x == x exactly and g = 0;
* a single-voxel scatterer has a closed-form solution;
* reciprocity: diag(m) A is complex-symmetric because K(r) = K(-r)^T;
* parity zeros and symmetry of the FFT symbol.
"""
import math

import numpy as np
import pytest

from oracle import kernel as K
from oracle import operator as op
from paper_1804_02297_amd import inputs as I


@pytest.mark.parametrize("n", [3, 4, 5, 8])
def test_fft_apply_equals_dense_sum(n):
    k = I.wavenumber_for(n)
    m = I.medium_random_complex(n, 10 + n)
    x = I.random_field(2, n, 20 + n)
    ref = op.apply_dense(n, k, m, x)
    got = op.apply_fft(n, k, m, x)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


def test_dense_sum_by_loops_tiny():
    """Independent loop form of Eq. (5) on n = 2 (8 points)."""
    n = 2
    k = 3.0
    h = K.grid_spacing(n)
    m = I.medium_random_complex(n, 1)
    x = I.random_field(1, n, 2)[0]
    pts = [(a, b, c) for a in range(n) for b in range(n) for c in range(n)]
    ref = np.array(x, copy=True)
    for i in pts:
        for j in pts:
            Kij = K.dyadic_tensor(np.array(i) - np.array(j), k, h)
            ref[(slice(None),) + i] += Kij @ (m[j] * x[(slice(None),) + j])
    got = op.apply_fft(n, k, m, x[None])[0]
    assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max()


def test_zero_contrast_is_identity():
    n = 6
    k = I.wavenumber_for(n)
    m = np.zeros((n, n, n), complex)
    x = I.random_field(2, n, 3)
    assert np.array_equal(op.apply_fft(n, k, m, x), x)
    Ei = I.plane_waves(n, k, [[1, 0, 0]], [[0, 0, 1]])
    assert not np.any(op.rhs_from_incident(n, k, m, Ei))


def test_single_voxel_closed_form():
    """m = m0 at j0 only: x_j0 = (I + m0 K(0))^-1 g_j0, x = g - m0 K(. - j0) x_j0."""
    n = 7
    k = I.wavenumber_for(n)
    h = K.grid_spacing(n)
    j0 = (2, 4, 3)
    m0 = 0.4 - 0.1j
    m = np.zeros((n, n, n), complex)
    m[j0] = m0
    g = I.random_field(1, n, 5)[0]
    xj0 = np.linalg.solve(np.eye(3) + m0 * K.dyadic_tensor(np.zeros(3), k, h), g[(slice(None),) + j0])
    x = np.array(g, copy=True)
    idx = op.grid_offsets(n)
    Kcol = K.dyadic_tensor(idx - np.array(j0), k, h)              # (n^3, 3, 3)
    x -= (m0 * (Kcol @ xj0)).T.reshape(3, n, n, n)
    x[(slice(None),) + j0] = xj0
    Ax = op.apply_fft(n, k, m, x[None])[0]
    assert np.abs(Ax - g).max() <= 1e-13 * np.abs(g).max()


def test_reciprocity_bilinear():
    n = 5
    k = I.wavenumber_for(n)
    m = I.medium_random_complex(n, 8)
    u = I.random_field(1, n, 9)[0]
    v = I.random_field(1, n, 10)[0]
    Au = op.apply_fft(n, k, m, u[None])[0]
    Av = op.apply_fft(n, k, m, v[None])[0]
    lhs = np.sum(v * m[None] * Au)
    rhs = np.sum(u * m[None] * Av)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_symbol_symmetry_and_parity_zeros():
    n = 6
    k = I.wavenumber_for(n)
    Kh = op.kernel_symbol(n, k)
    P = 2 * n
    scale = np.abs(Kh).max()
    assert np.allclose(Kh, Kh.transpose(1, 0, 2, 3, 4), atol=1e-13 * scale, rtol=0)
    q = np.arange(P)
    for a in range(3):
        for b in range(3):
            if a == b:
                continue
            for d in (a, b):
                sl = [slice(None)] * 3
                for qq in (0, n):
                    sl[d] = qq
                    assert np.abs(Kh[a, b][tuple(sl)]).max() <= 1e-13 * scale
    # evenness / oddness in each frequency: Khat(.., P - q_d, ..) = +-Khat
    neg = (-q) % P
    for a in range(3):
        for b in range(3):
            for d in range(3):
                sgn = -1.0 if (a != b and d in (a, b)) else 1.0
                flipped = np.take(Kh[a, b], neg, axis=d)
                assert np.abs(flipped - sgn * Kh[a, b]).max() <= 1e-13 * scale


def test_rhs_is_minus_convolution_of_incident():
    n = 5
    k = I.wavenumber_for(n)
    m = I.medium_single_bump(n, 2)
    d, p = I.random_direction_and_polarisation(3)
    Ei = I.plane_waves(n, k, [d], [p])
    g = op.rhs_from_incident(n, k, m, Ei)
    A = op.dense_matrix(n, k, m)
    ref = Ei.reshape(-1) - A @ Ei.reshape(-1)
    assert np.abs(g.reshape(-1) - ref).max() <= 1e-13 * np.abs(ref).max()
    # plane-wave sanity: transverse, unit amplitude
    assert abs(np.dot(d, p)) < 1e-14
    assert abs(np.linalg.norm(p) - 1) < 1e-14
    assert np.allclose(np.abs(Ei[0, np.argmax(np.abs(p))]), abs(p).max())
