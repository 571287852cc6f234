"""Nystrom operator A = I + K diag(m) and its FFT apply (oracle, FP64).
TEST INFRASTRUCTURE ONLY.

Paper: Eq. (5) (discrete equations), Eq. (6) (block form with diagonal m and
Toeplitz convolution matrices), Section 2 (FFT for the convolutions) and
Section 3.3 (FFT forward operator, O(N log N)).  In the dyadic form the
discrete system reads

  (A E)_i = E_i + sum_{j in I} K(i - j) m_j E_j ,    i in I = {1..n}^3,

where each K(i-j) is a 3x3 block (oracle.kernel.dyadic_tensor).

Functions
  dense_matrix / apply_dense : the definition, a literal double sum (small n).
  kernel_symbol              : FFT of the circulant embedding of K on P = 2n.
  apply_fft                  : zero-padded FFT convolution, the O(N log N) apply.
  rhs_from_incident          : g = -K * (m E^i) = E^i - A E^i (Eq. (4)).

Pins: apply_fft == apply_dense to 1e-13 on n <= 8 (brute force); m = 0 gives
A x == x exactly; a single-voxel scatterer has a closed-form solution.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from .kernel import dyadic_tensor, grid_spacing, kernel_table


def grid_offsets(n: int) -> np.ndarray:
    """All grid multi-indices (0-based) in C order, shape (n^3, 3)."""
    s = np.arange(n)
    return np.stack(np.meshgrid(s, s, s, indexing="ij"), axis=-1).reshape(-1, 3)


def dense_matrix(n: int, k: float, m: np.ndarray) -> np.ndarray:
    """A = I + K diag(m) as a dense (3n^3 x 3n^3) matrix, unknowns ordered [c, i1, i2, i3]."""
    h = grid_spacing(n)
    idx = grid_offsets(n)
    N = n ** 3
    d = idx[:, None, :] - idx[None, :, :]                     # i - j
    Kb = dyadic_tensor(d, k, h)                                # (N, N, 3, 3)
    Kmat = Kb.transpose(2, 0, 3, 1).reshape(3 * N, 3 * N)      # [(c,i),(c',j)]
    mv = np.tile(np.asarray(m, dtype=np.complex128).reshape(-1), 3)
    return np.eye(3 * N, dtype=np.complex128) + Kmat * mv[None, :]


def apply_dense(n: int, k: float, m: np.ndarray, x: np.ndarray) -> np.ndarray:
    """(A x) by the literal double sum; x of shape (..., 3, n, n, n)."""
    A = dense_matrix(n, k, m)
    xs = np.asarray(x, dtype=np.complex128)
    lead = xs.shape[:-4]
    flat = xs.reshape((-1, 3 * n ** 3))
    return (flat @ A.T).reshape(lead + (3, n, n, n))


def fft_size(n: int) -> int:
    """Padded length P = 2n of the circulant embedding."""
    return 2 * n


def embedded_kernel(n: int, k: float) -> np.ndarray:
    """Circulant embedding on P^3: K(r) at index r mod P for |r_d| <= n-1, zero at r_d = n.

    Shape (3, 3, P, P, P).
    """
    P = fft_size(n)
    T = kernel_table(n, k)                                     # (2n-1,)*3 + (3,3)
    emb = np.zeros((3, 3, P, P, P), dtype=np.complex128)
    s = np.arange(-(n - 1), n) % P
    emb[:, :, s[:, None, None], s[None, :, None], s[None, None, :]] = T.transpose(3, 4, 0, 1, 2)
    return emb


def kernel_symbol(n: int, k: float) -> np.ndarray:
    """Khat = unnormalised forward FFT of the embedding, shape (3, 3, P, P, P)."""
    return scipy.fft.fftn(embedded_kernel(n, k), axes=(-3, -2, -1))


def apply_fft(n: int, k: float, m: np.ndarray, x: np.ndarray, Khat=None) -> np.ndarray:
    """(A x) by zero-padded FFT convolution (Section 2; Section 3.3)."""
    P = fft_size(n)
    if Khat is None:
        Khat = kernel_symbol(n, k)
    xs = np.asarray(x, dtype=np.complex128)
    lead = xs.shape[:-4]
    xs = xs.reshape((-1, 3, n, n, n))
    out = np.empty_like(xs)
    mm = np.asarray(m, dtype=np.complex128)
    for r in range(xs.shape[0]):
        u = np.zeros((3, P, P, P), dtype=np.complex128)
        u[:, :n, :n, :n] = mm[None] * xs[r]
        uh = scipy.fft.fftn(u, axes=(-3, -2, -1))
        vh = np.einsum("abxyz,bxyz->axyz", Khat, uh)
        v = scipy.fft.ifftn(vh, axes=(-3, -2, -1))
        out[r] = xs[r] + v[:, :n, :n, :n]
    return out.reshape(lead + (3, n, n, n))


def rhs_from_incident(n: int, k: float, m: np.ndarray, Ei: np.ndarray, Khat=None) -> np.ndarray:
    """g = -K * (m E^i) = E^i - A E^i: right-hand side of the scattered-field equation (4)."""
    Ei = np.asarray(Ei, dtype=np.complex128)
    return Ei - apply_fft(n, k, m, Ei, Khat)
