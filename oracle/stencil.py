"""Local stencils alpha, beta (oracle, FP64).  TEST INFRASTRUCTURE ONLY.

Paper: Section 3.1 (Building the approximating sparse system) and Section 3.2
(Exploiting translational invariance to compute the stencils).

For a point i with neighbourhood tau_i = {j : |j - i|_inf <= 1} the rows of
Eq. (5) indexed by tau_i split into a local and a non-local part (Eqs. (7),
(8)).  In the dyadic form the non-local block is

  M = [ K(a - j) ]_{a in tau, j in tau^c}          (3|tau| x 3|tau^c|)

and the local block B = [ K(a - b) ]_{a, b in tau}.  A 3|tau| x 3 matrix alpha
with alpha^H M ~ 0 (Eq. (10)) turns the 3|tau| rows into three local rows
(Eq. (11)) with beta = B^H alpha (Eq. (12)).  Numerically alpha minimises
||alpha^H M||_F over alpha^H alpha = I, i.e. it holds the three left singular
vectors of M with the smallest singular values (end of Section 3.1).

Reading taken for the transpose: the paper writes alpha^T; a literal
transpose with alpha^T alpha = I is not a unitary constraint and has no SVD
solution, while "left singular vectors" is exact for the conjugate transpose.
So rows are alpha^H (...), alpha = U_min and beta = B^H alpha.

Translational invariance (Section 3.2): alpha, beta depend only on the
position class of i.  Per dimension the class is 'lo' (i_d = 1), 'hi'
(i_d = n) or 'in'; the 27 combinations are the interior, face, edge and vertex
classes.  Offsets s = j - i per dimension:

  class  tau_d        enlarged complement range
  in     {-1, 0, 1}   {-(n-2) .. n-2}
  lo     {0, 1}       {0 .. n-1}
  hi     {-1, 0}      {-(n-1) .. 0}

(the 'hi' rows mirror the paper's low-side examples).

Per-point medium-weighted fit (a project extension, not in the paper):
minimise sum_{j in tau^c} w_j^2 ||alpha^H K_{tau,j}||^2 over alpha^H alpha = I
with w_j = 1 + |m_{i+j}| / m0 on the 5^3 shell around i (98 offsets, m = 0
off the grid) and w_j = 1 elsewhere; it reduces to the class fit when m = 0 on
the shell.  Motivated by the dropped term alpha^H M diag(m) E of Eq. (9), whose
size grows with |m| (Section 4).

Gauge: S^-1 Q is invariant under alpha -> alpha X for invertible 3x3 X; the
gauge-fixed stencil alpha~ = alpha (alpha_centre)^-1 has the identity as its
centre block.

Pins: Ky Fan optimality ||alpha^H M||_F^2 = sum of the three smallest
sigma^2 and alpha^H alpha = I; the SVD stencil is at least as local as the
best blockdiag(gamma) stencil of Eq. (13); reflection / permutation relations
between the 27 classes; the weighted fit with unit weights equals the class
fit.
"""
from __future__ import annotations

import itertools

import numpy as np

from .kernel import dyadic_tensor, grid_spacing

LO, IN, HI = 0, 1, 2
CLASS_NAMES = ("lo", "in", "hi")


def point_class_dim(i: int, n: int) -> int:
    """Per-dimension class of a 1-based index i_d."""
    if i == 1:
        return LO
    if i == n:
        return HI
    return IN


def class_id(cls3) -> int:
    """Class index 9 c1 + 3 c2 + c3 in [0, 27); 13 is the interior class."""
    return 9 * cls3[0] + 3 * cls3[1] + cls3[2]


def class_of_point(i1: int, i2: int, i3: int, n: int) -> int:
    return class_id((point_class_dim(i1, n), point_class_dim(i2, n), point_class_dim(i3, n)))


def tau_1d(c: int):
    return {LO: [0, 1], IN: [-1, 0, 1], HI: [-1, 0]}[c]


def range_1d(c: int, n: int):
    return {LO: list(range(0, n)), IN: list(range(-(n - 2), n - 1)),
            HI: list(range(-(n - 1), 1))}[c]


def class_dims(kappa: int):
    return (kappa // 9, (kappa // 3) % 3, kappa % 3)


def tau_offsets(kappa: int) -> np.ndarray:
    """tau for class kappa as offsets, lexicographic with the last dimension fastest."""
    c = class_dims(kappa)
    return np.array(list(itertools.product(tau_1d(c[0]), tau_1d(c[1]), tau_1d(c[2]))), dtype=np.int64)


def complement_offsets(kappa: int, n: int) -> np.ndarray:
    """Enlarged complement tau^c of Section 3.2 as offsets."""
    c = class_dims(kappa)
    rng = [np.array(range_1d(cd, n)) for cd in c]
    g = np.stack(np.meshgrid(*rng, indexing="ij"), axis=-1).reshape(-1, 3)
    inside = np.all(np.abs(g) <= 1, axis=1)
    return g[~inside]


def nonlocal_block(kappa: int, n: int, k: float, cols=None) -> np.ndarray:
    """M = [K(a - j)]_{a in tau, j in tau^c}; rows (a, c), columns (j, c')."""
    h = grid_spacing(n)
    tau = tau_offsets(kappa)
    tc = complement_offsets(kappa, n) if cols is None else cols
    d = tau[:, None, :] - tc[None, :, :]
    Kb = dyadic_tensor(d, k, h)                       # (|tau|, |tc|, 3, 3)
    return Kb.transpose(0, 2, 1, 3).reshape(3 * len(tau), 3 * len(tc))


def local_block(kappa: int, n: int, k: float) -> np.ndarray:
    """B = [K(a - b)]_{a, b in tau} (includes the self term on the diagonal)."""
    h = grid_spacing(n)
    tau = tau_offsets(kappa)
    d = tau[:, None, :] - tau[None, :, :]
    Kb = dyadic_tensor(d, k, h)
    return Kb.transpose(0, 2, 1, 3).reshape(3 * len(tau), 3 * len(tau))


def fit_class(kappa: int, n: int, k: float):
    """alpha = three smallest left singular vectors of M (thin SVD), beta = B^H alpha.

    Returns (alpha, beta, sigma) with sigma the singular values of M, ascending.
    """
    M = nonlocal_block(kappa, n, k)
    U, s, _ = np.linalg.svd(M, full_matrices=False)
    order = np.argsort(s)
    alpha = U[:, order[:3]]
    beta = local_block(kappa, n, k).conj().T @ alpha
    return alpha, beta, s[order]


def fit_all_classes(n: int, k: float):
    """The 27 class stencils: lists alpha[kappa], beta[kappa], sigma[kappa]."""
    if n < 4:
        # n = 3: the interior class has an empty complement (any alpha is optimal)
        raise ValueError("class fit needs n >= 4")
    out = [fit_class(kappa, n, k) for kappa in range(27)]
    return [o[0] for o in out], [o[1] for o in out], [o[2] for o in out]


def projector(alpha: np.ndarray) -> np.ndarray:
    """Orthogonal projector onto span(alpha)."""
    q, _ = np.linalg.qr(alpha)
    return q @ q.conj().T


def gamma_stencil(kappa: int, n: int, k: float):
    """Best scalar stencil gamma for the block-diagonal alpha of Eq. (13).

    gamma minimises ||gamma^H [G, G^1, G^2, G^3]_{tau, tau^c}|| over unit
    gamma (Section 3.1: G and its derivatives solve Helmholtz off the origin).
    Returns alpha = blockdiag(gamma, gamma, gamma) in the (a, c) row order.
    """
    h = grid_spacing(n)
    tau = tau_offsets(kappa)
    tc = complement_offsets(kappa, n)
    x = h * (tau[:, None, :] - tc[None, :, :]).astype(np.float64)
    R = np.sqrt(np.sum(x * x, axis=-1))
    G = np.exp(1j * k * R) / (4 * np.pi * R)
    dG = G * (1j * k - 1.0 / R)                      # dG/dR
    blocks = [G] + [dG * x[..., d] / R for d in range(3)]
    Msc = np.concatenate(blocks, axis=1)
    U, s, _ = np.linalg.svd(Msc, full_matrices=False)
    g = U[:, np.argmin(s)]
    alpha = np.zeros((3 * len(tau), 3), dtype=np.complex128)
    for c in range(3):
        alpha[c::3, c] = g
    return alpha


SHELL_RADIUS = 2


def shell_offsets() -> np.ndarray:
    """Offsets of the 5^3 patch outside tau: 98 points."""
    s = np.arange(-SHELL_RADIUS, SHELL_RADIUS + 1)
    g = np.stack(np.meshgrid(s, s, s, indexing="ij"), axis=-1).reshape(-1, 3)
    return g[np.any(np.abs(g) > 1, axis=1)]


def shell_weights(m: np.ndarray, i0, m0: float):
    """w_j = 1 + |m_{i+j}| / m0 on the shell (m = 0 off the grid).  i0 is 0-based."""
    n = m.shape[0]
    sh = shell_offsets()
    w = np.ones(len(sh))
    for t, s in enumerate(sh):
        p = np.asarray(i0) + s
        if np.all(p >= 0) and np.all(p < n):
            w[t] = 1.0 + abs(m[tuple(p)]) / m0
    return sh, w


def fit_point_weighted(m: np.ndarray, i0, k: float, m0: float = 0.1):
    """Medium-weighted per-point fit (project extension): SVD of M diag(w).

    i0 is the 0-based grid index of the point.  Returns (alpha, beta, sigma).
    """
    n = m.shape[0]
    kappa = class_of_point(i0[0] + 1, i0[1] + 1, i0[2] + 1, n)
    tc = complement_offsets(kappa, n)
    sh, wsh = shell_weights(m, i0, m0)
    w = np.ones(len(tc))
    lookup = {tuple(s): t for t, s in enumerate(sh)}
    for t, s in enumerate(tc):
        q = lookup.get(tuple(s))
        if q is not None:
            w[t] = wsh[q]
    M = nonlocal_block(kappa, n, k, cols=tc)
    Mw = M * np.repeat(w, 3)[None, :]
    U, s, _ = np.linalg.svd(Mw, full_matrices=False)
    order = np.argsort(s)
    alpha = U[:, order[:3]]
    beta = local_block(kappa, n, k).conj().T @ alpha
    return alpha, beta, s[order]


def weighted_gram(m: np.ndarray, i0, k: float, m0: float = 0.1) -> np.ndarray:
    """Gram_i = M diag(w^2) M^H of the weighted per-point objective."""
    n = m.shape[0]
    kappa = class_of_point(i0[0] + 1, i0[1] + 1, i0[2] + 1, n)
    tc = complement_offsets(kappa, n)
    sh, wsh = shell_weights(m, i0, m0)
    lookup = {tuple(s): t for t, s in enumerate(sh)}
    w = np.array([wsh[lookup[tuple(s)]] if tuple(s) in lookup else 1.0 for s in tc])
    M = nonlocal_block(kappa, n, k, cols=tc)
    Mw = M * np.repeat(w, 3)[None, :]
    return Mw @ Mw.conj().T


def interior_gram_parts(n: int, k: float):
    """The pieces of every interior point's weighted Gram.

    The weighted objective sums w_j^2 K_{tau,j} K_{tau,j}^H over the columns j
    of the complement, and w_j = 1 off the 5^3 shell, so

      Gram_i = M M^H + sum_{s in shell} (w_s^2 - 1) K_{tau,s} K_{tau,s}^H

    with M the interior class's non-local block.  Returns (M M^H, shell
    offsets, [K_{tau,s} K_{tau,s}^H for each shell offset]).
    """
    M = nonlocal_block(13, n, k)
    sh = shell_offsets()
    Ks = nonlocal_block(13, n, k, cols=sh)              # 81 x 3*98
    H = [Ks[:, 3 * t:3 * t + 3] @ Ks[:, 3 * t:3 * t + 3].conj().T for t in range(len(sh))]
    return M @ M.conj().T, sh, H


def weighted_gram_from_parts(parts, m: np.ndarray, i0, m0: float = 0.1) -> np.ndarray:
    """weighted_gram of an interior point from interior_gram_parts."""
    G0, sh, H = parts
    sh2, w = shell_weights(m, i0, m0)
    assert np.array_equal(sh, sh2)
    G = G0.copy()
    for t in range(len(sh)):
        G += (w[t] ** 2 - 1.0) * H[t]
    return G


# A predicted stencil is accepted only when it is more local than the class
# stencil on the point's own objective by more than this relative amount, so
# that a prediction equal to the class stencil falls back to the exact fit.
ACCEPT_RTOL = 1e-9


def locality_ratio(alpha_hat: np.ndarray, gram: np.ndarray, alpha_class: np.ndarray) -> float:
    """rho = tr(Q^H Gram Q) / tr(Q_c^H Gram Q_c) over the spans of the prediction and the class stencil."""
    return locality(alpha_hat, gram) / locality(alpha_class, gram)


def accept_prediction(rho: float) -> bool:
    """The acceptance rule of the learned fit: rho < 1 - ACCEPT_RTOL."""
    return rho < 1.0 - ACCEPT_RTOL


def centre_index(kappa: int) -> int:
    """Position of offset (0,0,0) in tau_offsets(kappa)."""
    tau = tau_offsets(kappa)
    return int(np.nonzero(np.all(tau == 0, axis=1))[0][0])


def gauge_fix(alpha: np.ndarray, kappa: int = 13) -> np.ndarray:
    """alpha~ = alpha (alpha_centre)^-1: centre 3x3 block becomes the identity."""
    c = centre_index(kappa)
    A0 = alpha[3 * c:3 * c + 3, :]
    return alpha @ np.linalg.inv(A0)


def gauge_condition(alpha: np.ndarray, kappa: int = 13) -> float:
    """|A0|_F |A0^-1|_F of the centre block; the gauge is used only when <= 1e6."""
    c = centre_index(kappa)
    A0 = alpha[3 * c:3 * c + 3, :]
    return float(np.linalg.norm(A0) * np.linalg.norm(np.linalg.inv(A0)))


def locality(alpha: np.ndarray, gram: np.ndarray) -> float:
    """tr(q^H Gram q) with q an orthonormal basis of span(alpha)."""
    q, _ = np.linalg.qr(alpha)
    return float(np.real(np.trace(q.conj().T @ gram @ q)))
