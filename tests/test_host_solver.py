"""The library's host multifrontal solver against SciPy's sparse LU (CPU only).

S comes from the oracle (class stencils, Eq. (11) rows) and is handed to the
library in its row layout [n^3][3][27][3]; the solve of the library must
equal scipy.sparse.linalg.spsolve on the same matrix to rounding.
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import sparse as osp
from oracle import stencil as ost
from paper_1804_02297_amd import binding
from paper_1804_02297_amd import inputs as I


def csr_to_rows(S, n):
    """Oracle CSR (rows r*N + p, cols c*N + q) -> [n^3][3][27][3] slot layout."""
    N = n ** 3
    rows = np.zeros((N, 3, 27, 3), np.complex128)
    S = S.tocoo()
    r, p = np.divmod(S.row, N)
    c, q = np.divmod(S.col, N)
    pi = np.stack(np.unravel_index(p, (n, n, n)), 1)
    qi = np.stack(np.unravel_index(q, (n, n, n)), 1)
    s = qi - pi
    assert np.abs(s).max() <= 1
    slot = 9 * (s[:, 0] + 1) + 3 * (s[:, 1] + 1) + (s[:, 2] + 1)
    np.add.at(rows, (p, r, slot, c), S.data)
    return rows


pytestmark = pytest.mark.skipif(not os.path.exists(binding.LIB_PATH), reason="library not built")


@pytest.mark.parametrize("n,seed", [(4, 0), (5, 1), (8, 2), (11, 3)])
def test_host_multifrontal_matches_spsolve(n, seed):
    k = I.wavenumber_for(n)
    m = I.medium_bumps(n, seed)
    al, be, _ = ost.fit_all_classes(n, k)
    S, Q = osp.assemble(n, m, al, be)
    rows = csr_to_rows(S, n)
    sp = binding.SparseHost(n, rows)
    b = I.random_field(2, n, 50 + seed)
    x = sp.solve(b)
    ref = np.stack([spla.spsolve(S.tocsc(), bb.reshape(-1)).reshape(3, n, n, n) for bb in b])
    assert np.abs(x - ref).max() <= 1e-10 * np.abs(ref).max()
    # residual check independent of scipy's solution
    res = np.stack([(S @ xx.reshape(-1) - bb.reshape(-1)) for xx, bb in zip(x, b)])
    assert np.abs(res).max() <= 1e-10 * np.abs(b).max()
    info = sp.info()
    assert info["bytes"] > 0 and info["flops"] > 0


@pytest.mark.parametrize("nrhs", [3, 5, 9, 13, 34])
def test_host_block_solve_matches_single(nrhs):
    """The block (many right-hand side) solve equals one-at-a-time solves."""
    n = 7
    k = I.wavenumber_for(n)
    m = I.medium_bumps(n, 4)
    al, be, _ = ost.fit_all_classes(n, k)
    S, _ = osp.assemble(n, m, al, be)
    sp = binding.SparseHost(n, csr_to_rows(S, n))
    b = I.random_field(nrhs, n, 70 + nrhs)
    x = sp.solve(b)
    for r in sorted({0, nrhs // 2, nrhs - 1}):
        one = sp.solve(b[r:r + 1])[0]
        assert np.abs(x[r] - one).max() <= 1e-12 * np.abs(one).max(), r
    res = np.stack([(S @ xx.reshape(-1) - bb.reshape(-1)) for xx, bb in zip(x, b)])
    assert np.abs(res).max() <= 1e-10 * np.abs(b).max()


def test_host_solver_random_matrix_same_pattern():
    """A random matrix on the 27-point pattern with a strong diagonal."""
    n = 6
    g = np.random.default_rng(0)
    N = n ** 3
    rows = np.zeros((N, 3, 27, 3), np.complex128)
    for p in range(N):
        i = np.unravel_index(p, (n, n, n))
        for slot in range(27):
            s = np.array([slot // 9 - 1, (slot // 3) % 3 - 1, slot % 3 - 1])
            j = np.array(i) + s
            if np.all(j >= 0) and np.all(j < n):
                rows[p, :, slot, :] = g.standard_normal((3, 3)) + 1j * g.standard_normal((3, 3))
        rows[p, :, 13, :] += 20 * np.eye(3)
    sp = binding.SparseHost(n, rows)
    b = I.random_field(1, n, 9)
    x = sp.solve(b)
    # rebuild S densely and check the residual
    S = np.zeros((3 * N, 3 * N), np.complex128)
    for p in range(N):
        i = np.unravel_index(p, (n, n, n))
        for slot in range(27):
            s = np.array([slot // 9 - 1, (slot // 3) % 3 - 1, slot % 3 - 1])
            j = np.array(i) + s
            if np.all(j >= 0) and np.all(j < n):
                q = np.ravel_multi_index(tuple(j), (n, n, n))
                for r in range(3):
                    for c in range(3):
                        S[r * N + p, c * N + q] = rows[p, r, slot, c]
    res = S @ x.reshape(-1) - b.reshape(-1)
    assert np.abs(res).max() <= 1e-11 * np.abs(b).max()


def test_memory_cap_is_enforced():
    n = 8
    rows = np.zeros((n ** 3, 3, 27, 3), np.complex128)
    rows[:, :, 13, :] = np.eye(3)
    with pytest.raises(binding.LSError) as e:
        binding.SparseHost(n, rows, host_mem_cap=1000)
    assert e.value.code == -5


@pytest.mark.parametrize("nrhs", [1, 6])
def test_host_fp32_factor_is_single_precision_solve(nrhs):
    """complex64 factor: the solve equals the complex128 one to single-precision
    accuracy (times the conditioning of S), and its block solve equals its
    one-at-a-time solves."""
    n = 7
    k = I.wavenumber_for(n)
    m = I.medium_bumps(n, 6)
    al, be, _ = ost.fit_all_classes(n, k)
    S, _ = osp.assemble(n, m, al, be)
    rows = csr_to_rows(S, n)
    sp64 = binding.SparseHost(n, rows)
    sp32 = binding.SparseHost(n, rows, prec="c64")
    assert sp32.info()["bytes"] * 2 == sp64.info()["bytes"]
    b = I.random_field(nrhs, n, 90 + nrhs)
    x64 = sp64.solve(b)
    x32 = sp32.solve(b)
    assert x32.dtype == np.complex128
    rel = np.abs(x32 - x64).max() / np.abs(x64).max()
    assert 1e-9 < rel <= 1e-4, rel                 # single, not double, precision
    if nrhs > 1:
        one = sp32.solve(b[1:2])[0]
        assert np.abs(x32[1] - one).max() <= 1e-5 * np.abs(one).max()
