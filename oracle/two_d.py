"""The paper's 2-D variant (oracle, FP64).  TEST INFRASTRUCTURE ONLY.

Paper: Section 2 notes that the scattered-field equation holds in 2-D with G
the 2-D Helmholtz kernel; Section 3.3 gives the 2-D costs; Section 4 the 2-D
examples (n = 119 .. 959, six points per wavelength, GMRES(20) to 1e-6,
E^i = (0, e^{i k x_1})).  The field has two components E = (E^1, E^2) on the
n x n grid of the unit square, h = 1/(n+1), x_i = i h, arrays [c, i1, i2].

  G(x) = (i/4) H_0^(1)(k |x|),     dG/dx_d = -(i k / 4) H_1^(1)(k |x|) x_d / |x|

The discrete equations (component d = 1, 2) are the 2-D form of the paper's
Section 2 equations:

  E^d_i + k^2 sum_j G_ij m_j E^d_j + sum_j G^d_ij (p^1_j E^1_j + p^2_j E^2_j) = g^d_i

with G_ij = h^2 G(x_i - x_j), G^d_ij = h^2 dG/dx_d (x_i - x_j) off the diagonal.

Readings (the same ones as for the 3-D paper form):
  * self weight of G: its integral over the disc of area h^2 about 0,
        (i pi a / (2k)) H_1^(1)(k a) - 1/k^2,   a = h / sqrt(pi);
    self weight of G^d: 0 (an odd kernel).
  * p^d = central difference of m (m = 0 off the grid) over 2h, divided by 1 - m.
  * stencils (Section 3.1): alpha^H for the paper's alpha^T; alpha holds the
    two left singular vectors of
        M = [[k^2 G, 0, G^1], [0, k^2 G, G^2]]   over tau x tau^c
    with the smallest singular values, beta = B^H alpha with B the same
    block over tau x tau (self weights on its diagonal).  Rows of alpha are
    (a, c) -> 2 t + c, rows of beta (a, f) -> 3 t + f, f = 0, 1 for m E^f and
    f = 2 for p.E.
  * classes (Section 3.2 in two dimensions): per dimension lo (i_d = 1),
    in, hi (i_d = n); tau_d = {0, 1}, {-1, 0, 1}, {-1, 0} and the enlarged
    complement ranges {0 .. n-1}, {-(n-2) .. n-2}, {-(n-1) .. 0}; class
    3 c1 + c2, the interior class is 4.

Rows of S and Q for point i of class kappa and neighbour a = tau[t]:
  Q[(r, i), (c, i+a)] = conj(alpha[2t+c, r])
  S[(r, i), (c, i+a)] = conj(alpha[2t+c, r]) + conj(beta[3t+c, r]) m_{i+a}
                        + conj(beta[3t+2, r]) p^c_{i+a}

Pins (tests/test_oracle_two_d.py): the FFT apply equals the double sum; G
has the fundamental solution's logarithmic singularity, solves the Helmholtz
equation away from 0 and has the outgoing far-field asymptotics; dG equals a
finite difference of G; the self weight equals a quadrature over the disc;
p converges at second order; m = 0 gives A x = x; the fit attains the Ky
Fan minimum and the lo / hi classes are mirror images; the solution
satisfies Gauss's law div((1 - m) E) = 0 at second order (a wrong sign or
index in the G^d term breaks it); preconditioned GMRES needs few iterations.
The field inside a small homogeneous cylinder is the static 2 E0 / (eps + 1),
eps = 1 - m, within 2 % (tests/test_oracle_physics.py; the central difference
of m over the jump leaves about 1 % as h -> 0).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.fft
import scipy.sparse
import scipy.special

from .stencil import point_class_dim, range_1d, tau_1d


def grid_spacing(n: int) -> float:
    return 1.0 / (n + 1)


def G2(R, k: float):
    """(i/4) H_0^(1)(k R), R > 0."""
    return 0.25j * scipy.special.hankel1(0, k * np.asarray(R, dtype=np.float64))


def dG2(x: np.ndarray, k: float) -> np.ndarray:
    """grad G at points x (..., 2), x != 0: -(i k/4) H_1^(1)(k R) x / R."""
    x = np.asarray(x, dtype=np.float64)
    R = np.sqrt(np.sum(x * x, axis=-1))
    return (-0.25j * k * scipy.special.hankel1(1, k * R) / R)[..., None] * x


def disc_integral_G2(k: float, h: float) -> complex:
    """int of G over the disc of area h^2 about 0: (i pi a/(2k)) H_1^(1)(k a) - 1/k^2."""
    a = h / math.sqrt(math.pi)
    return complex(0.5j * math.pi * a / k * scipy.special.hankel1(1, k * a) - 1.0 / k ** 2)


def gradient_p2(n: int, m: np.ndarray) -> np.ndarray:
    """p^d = (dm/dx_d) / (1 - m) by central differences, shape (2, n, n)."""
    h = grid_spacing(n)
    m = np.asarray(m, dtype=np.complex128)
    mp = np.zeros((n + 2, n + 2), dtype=np.complex128)
    mp[1:-1, 1:-1] = m
    c = slice(1, n + 1)
    p = np.stack([(mp[2:, c] - mp[:-2, c]) / (2 * h), (mp[c, 2:] - mp[c, :-2]) / (2 * h)])
    return p / (1.0 - m)[None]


def weights_at(r: np.ndarray, n: int, k: float) -> np.ndarray:
    """(G, G^1, G^2) weights for integer offsets r (..., 2), self weights at r = 0; shape (3, ...)."""
    h = grid_spacing(n)
    x = h * np.asarray(r, dtype=np.float64)
    R = np.sqrt(np.sum(x * x, axis=-1))
    zero = R == 0.0
    xs = np.where(zero[..., None], 1.0, x)
    Rs = np.where(zero, 1.0, R)
    out = np.empty((3,) + R.shape, dtype=np.complex128)
    out[0] = h ** 2 * G2(Rs, k)
    out[1:] = h ** 2 * np.moveaxis(dG2(xs, k), -1, 0)
    out[0][zero] = disc_integral_G2(k, h)
    out[1][zero] = 0.0
    out[2][zero] = 0.0
    return out


def weights2(n: int, k: float) -> np.ndarray:
    """(G, G^1, G^2) for offsets in [-(n-1), n-1]^2, shape (3, 2n-1, 2n-1)."""
    s = np.arange(-(n - 1), n)
    return weights_at(np.stack(np.meshgrid(s, s, indexing="ij"), axis=-1), n, k)


def apply_dense2(n: int, k: float, m: np.ndarray, x: np.ndarray) -> np.ndarray:
    """The definition, literal double sums over i and j (small n)."""
    W = weights2(n, k)
    p = gradient_p2(n, m)
    m = np.asarray(m, dtype=np.complex128)
    x = np.asarray(x, dtype=np.complex128).reshape(2, n, n)
    u = m[None] * x
    w = p[0] * x[0] + p[1] * x[1]
    y = x.copy()
    for i1 in range(n):
        for i2 in range(n):
            for j1 in range(n):
                for j2 in range(n):
                    r1, r2 = i1 - j1 + n - 1, i2 - j2 + n - 1
                    for d in range(2):
                        y[d, i1, i2] += k * k * W[0, r1, r2] * u[d, j1, j2] + W[1 + d, r1, r2] * w[j1, j2]
    return y


def symbol2(n: int, k: float) -> np.ndarray:
    """FFT of the circulant embedding (P = 2n) of (k^2 G, G^1, G^2), shape (3, P, P)."""
    P = 2 * n
    W = weights2(n, k)
    W[0] *= k * k
    emb = np.zeros((3, P, P), dtype=np.complex128)
    s = np.arange(-(n - 1), n) % P
    emb[:, s[:, None], s[None, :]] = W
    return scipy.fft.fftn(emb, axes=(-2, -1))


def apply_fft2(n: int, k: float, m: np.ndarray, x: np.ndarray, sym=None) -> np.ndarray:
    """A x by zero-padded FFT convolution: transforms of m E^1, m E^2, p.E, the 2x3 multiply, inverse."""
    P = 2 * n
    if sym is None:
        sym = symbol2(n, k)
    p = gradient_p2(n, m)
    mm = np.asarray(m, dtype=np.complex128)
    xs = np.asarray(x, dtype=np.complex128)
    lead = xs.shape[:-3]
    xs = xs.reshape((-1, 2, n, n))
    out = np.empty_like(xs)
    for r in range(xs.shape[0]):
        u = np.zeros((3, P, P), dtype=np.complex128)
        u[:2, :n, :n] = mm[None] * xs[r]
        u[2, :n, :n] = p[0] * xs[r, 0] + p[1] * xs[r, 1]
        uh = scipy.fft.fftn(u, axes=(-2, -1))
        vh = sym[0][None] * uh[:2] + sym[1:] * uh[2][None]
        v = scipy.fft.ifftn(vh, axes=(-2, -1))
        out[r] = xs[r] + v[:, :n, :n]
    return out.reshape(lead + (2, n, n))


def rhs2(n: int, k: float, m: np.ndarray, Ei: np.ndarray, sym=None) -> np.ndarray:
    """g = E^i - A E^i, the right-hand side for the scattered field."""
    Ei = np.asarray(Ei, dtype=np.complex128)
    return Ei - apply_fft2(n, k, m, Ei, sym)


# --- stencils (Sections 3.1, 3.2 in two dimensions) ---

def class_of_point2(i1: int, i2: int, n: int) -> int:
    """Class 3 c1 + c2 of the 1-based point (i1, i2)."""
    return 3 * point_class_dim(i1, n) + point_class_dim(i2, n)


def tau_offsets2(kappa: int) -> np.ndarray:
    return np.array(list(itertools.product(tau_1d(kappa // 3), tau_1d(kappa % 3))), dtype=np.int64)


def complement_offsets2(kappa: int, n: int) -> np.ndarray:
    rng = [np.array(range_1d(kappa // 3, n)), np.array(range_1d(kappa % 3, n))]
    g = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 2)
    return g[~np.all(np.abs(g) <= 1, axis=1)]


def coupling_block2(rows: np.ndarray, cols: np.ndarray, n: int, k: float) -> np.ndarray:
    """[[k^2 G, 0, G^1], [0, k^2 G, G^2]] over rows x cols: rows (a, c) -> 2a + c, columns (j, f) -> 3j + f."""
    W = weights_at(rows[:, None, :] - cols[None, :, :], n, k)        # (3, |rows|, |cols|)
    out = np.zeros((len(rows), 2, len(cols), 3), dtype=np.complex128)
    for c in range(2):
        out[:, c, :, c] = k * k * W[0]
        out[:, c, :, 2] = W[1 + c]
    return out.reshape(2 * len(rows), 3 * len(cols))


def fit_class2(kappa: int, n: int, k: float):
    """alpha = two smallest left singular vectors of M, beta = B^H alpha; sigma ascending."""
    tau = tau_offsets2(kappa)
    M = coupling_block2(tau, complement_offsets2(kappa, n), n, k)
    U, s, _ = np.linalg.svd(M, full_matrices=False)
    order = np.argsort(s)
    alpha = U[:, order[:2]]
    beta = coupling_block2(tau, tau, n, k).conj().T @ alpha
    return alpha, beta, s[order]


def fit_all_classes2(n: int, k: float):
    if n < 4:
        raise ValueError("class fit needs n >= 4")
    out = [fit_class2(kappa, n, k) for kappa in range(9)]
    return [o[0] for o in out], [o[1] for o in out], [o[2] for o in out]


def assemble2(n: int, m: np.ndarray, alphas, betas):
    """S and Q (CSR, 2n^2 x 2n^2), rows [r, i1, i2], unknowns [c, i1, i2]."""
    N = n * n
    mm = np.asarray(m, dtype=np.complex128)
    p = gradient_p2(n, mm)
    rows, cols, sv, qv = [], [], [], []
    for i1 in range(n):
        for i2 in range(n):
            kappa = class_of_point2(i1 + 1, i2 + 1, n)
            alpha, beta = alphas[kappa], betas[kappa]
            for t, a in enumerate(tau_offsets2(kappa)):
                j1, j2 = i1 + a[0], i2 + a[1]
                for r in range(2):
                    for c in range(2):
                        qa = np.conj(alpha[2 * t + c, r])
                        rows.append(r * N + i1 * n + i2)
                        cols.append(c * N + j1 * n + j2)
                        qv.append(qa)
                        sv.append(qa + np.conj(beta[3 * t + c, r]) * mm[j1, j2]
                                  + np.conj(beta[3 * t + 2, r]) * p[c, j1, j2])
    shape = (2 * N, 2 * N)
    S = scipy.sparse.csr_matrix((np.array(sv), (rows, cols)), shape=shape)
    Q = scipy.sparse.csr_matrix((np.array(qv), (rows, cols)), shape=shape)
    return S, Q

