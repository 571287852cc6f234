"""The GPU multifrontal factor and solves of S.

Small grids: S comes from the oracle (class stencils, Eq. (11) rows, Section
3.1) in the library's row layout and the GPU solve must equal SciPy's sparse
LU solve: a complex128 factor to 1e-10 of the solution's size (the host
factor's bar), a complex64 factor to single precision.  Larger grids, where
splu is too slow for a test: the residual ||S x - b|| / ||b|| with S applied
from its rows by a plain numpy stencil sum (a property that holds at any
size).  Solves of up to four right-hand sides take the matrix-vector path
and equal one-at-a-time solves bitwise; larger blocks take the MFMA path,
bitwise equal among themselves (every right-hand side takes the same
arithmetic) and equal to the single solves to rounding (another summation
order).
"""
import ctypes

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import sparse as osp
from oracle import stencil as ost
from paper_1804_02297_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _rows_from_csr(S, n):
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


def _rows_matvec(rows, x, n):
    """S x from the rows: y[r](p) = sum over slots s and components c of
    rows[p, r, s, c] x[c](p + offset(s)), neighbours outside the grid skipped."""
    R = rows.reshape(n, n, n, 3, 27, 3)
    xp = np.zeros((3, n + 2, n + 2, n + 2), np.complex128)
    xp[:, 1:-1, 1:-1, 1:-1] = x
    y = np.zeros((3, n, n, n), np.complex128)
    for slot in range(27):
        s1, s2, s3 = slot // 9 - 1, (slot // 3) % 3 - 1, slot % 3 - 1
        xs = xp[:, 1 + s1:1 + s1 + n, 1 + s2:1 + s2 + n, 1 + s3:1 + s3 + n]
        for r in range(3):
            for c in range(3):
                y[r] += R[:, :, :, r, slot, c] * xs[c]
    return y


def _oracle_system(n, seed):
    k = I.wavenumber_for(n)
    m = I.medium_bumps(n, seed)
    al, be, _ = ost.fit_all_classes(n, k)
    S, _ = osp.assemble(n, m, al, be)
    return S.tocsc(), _rows_from_csr(S, n)


@pytest.mark.parametrize("n,seed", [(4, 0), (5, 1), (8, 2), (11, 3), (16, 4)])
def test_gpu_factor_matches_splu(lib, n, seed):
    """One leaf (n = 4: a single 192-unknown front, four tiles), two levels
    (n = 5), deeper trees with ragged last tiles (n = 8, 11, 16)."""
    from paper_1804_02297_amd.binding import SparseGpu
    S, rows = _oracle_system(n, seed)
    b = I.random_field(3, n, 60 + seed)
    lu = spla.splu(S)
    ref = np.stack([lu.solve(bb.reshape(-1)).reshape(3, n, n, n) for bb in b])
    print(f"n={n} seed={seed}", flush=True)
    sp = SparseGpu(n, rows, prec="c128")
    x = sp.solve(_dev(b)).cpu().numpy()
    err = np.abs(x - ref).max() / np.abs(ref).max()
    res = max(np.abs(S @ xx.reshape(-1) - bb.reshape(-1)).max() for xx, bb in zip(x, b)) / np.abs(b).max()
    print(f"  c128 err {err:.2e} resid {res:.2e}", flush=True)
    assert err <= 1e-10 and res <= 1e-10
    b64 = sp.info()["bytes"]
    sp.close()
    sp = SparseGpu(n, rows, prec="c64")
    x = sp.solve(_dev(b)).cpu().numpy()
    rel = np.linalg.norm(x - ref) / np.linalg.norm(ref)
    print(f"  c64 rel err {rel:.2e}", flush=True)
    assert rel <= 1e-4
    assert sp.info()["bytes"] * 2 == b64
    sp.close()


def test_gpu_factor_equals_host_factor(lib):
    """Both factorisations of the same S solve to the same field (FP64)."""
    from paper_1804_02297_amd.binding import SparseGpu, SparseHost
    n = 12
    _, rows = _oracle_system(n, 5)
    b = I.random_field(2, n, 71)
    xh = SparseHost(n, rows).solve(b)
    xg = SparseGpu(n, rows).solve(_dev(b)).cpu().numpy()
    assert np.abs(xg - xh).max() <= 1e-12 * np.abs(xh).max()


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_block_solve_equals_single_solves(lib, prec):
    """nrhs across the 64-rhs workgroup chunks of the solve kernels, ragged
    last chunk: bitwise within each path (matrix-vector up to four rhs, MFMA
    above), and the two paths equal to rounding."""
    from paper_1804_02297_amd.binding import SparseGpu
    n = 9
    _, rows = _oracle_system(n, 6)
    sp = SparseGpu(n, rows, prec=prec)
    b = I.random_field(70, n, 80)
    single = np.stack([sp.solve(_dev(b[i:i + 1])).cpu().numpy()[0] for i in range(len(b))])
    for nr in (2, 3, 4):
        assert np.array_equal(sp.solve(_dev(b[:nr])).cpu().numpy(), single[:nr]), nr
    full = sp.solve(_dev(b)).cpu().numpy()
    tol = 1e-12 if prec == "c128" else 2e-5
    assert np.abs(full - single).max() <= tol * np.abs(single).max()
    for nr in (5, 17, 33, 64, 65):
        xb = sp.solve(_dev(b[:nr])).cpu().numpy()
        assert np.array_equal(xb, full[:nr]), nr


@pytest.mark.parametrize("n", [32, 48])
def test_gpu_factor_residual_at_larger_grids(lib, n):
    """S from the GPU stencil fit (the plan's rows); residual from the rows."""
    from paper_1804_02297_amd.binding import Plan
    k = I.wavenumber_for(n)
    m = I.medium_bumps(n, 1)
    plan = Plan(n, k, _dev(m), max_rhs=1)
    plan.stencil_fit()
    rows = plan.rows()
    b = I.random_field(2, n, 90)
    for prec, bar in (("c128", 1e-10), ("c64", 1e-4)):
        print(f"n={n} {prec}", flush=True)
        t = plan.factor_gpu(prec)
        from paper_1804_02297_amd.binding import SparseGpu
        sp = SparseGpu(n, rows, prec=prec)
        x = sp.solve(_dev(b)).cpu().numpy()
        res = max(np.linalg.norm(_rows_matvec(rows, xx, n) - bb) / np.linalg.norm(bb) for xx, bb in zip(x, b))
        print(f"  factor {t:.3f} s, residual {res:.2e}", flush=True)
        assert res <= bar
        sp.close()


@pytest.mark.parametrize("factor_prec", ["c128", "c64"])
def test_plan_solve_with_gpu_factor(lib, factor_prec):
    """FGMRES with the GPU factor reaches the FP64 bar (oracle residual) in the
    same number of iterations as with the host factor of the same precision."""
    from oracle import operator as oop
    from paper_1804_02297_amd.binding import Plan
    n = 12
    k = I.wavenumber_for(n)
    m = I.medium_bumps(n, 1)
    dirs, pols = I.fibonacci_incident_set(2)
    Ei = I.plane_waves(n, k, dirs, pols)
    plan = Plan(n, k, _dev(m), max_rhs=4)
    g = plan.rhs_from_incident(_dev(Ei))
    plan.stencil_fit()
    plan.factor(factor_prec)
    _, info_h, st = plan.solve(g, tol=1e-8, restart=30, prec="mixed")
    assert st == 0
    plan.factor_gpu(factor_prec)
    x, info, st = plan.solve(g, tol=1e-8, restart=30, prec="mixed")
    assert st == 0, info
    gh = g.cpu().numpy()
    r = gh - oop.apply_fft(n, k, m, x.cpu().numpy())
    rr = np.linalg.norm(r.reshape(len(gh), -1), axis=1) / np.linalg.norm(gh.reshape(len(gh), -1), axis=1)
    print(factor_prec, [i["iters"] for i in info_h], [i["iters"] for i in info], rr, flush=True)
    assert rr.max() <= 1e-8
    assert [i["iters"] for i in info] == [i["iters"] for i in info_h]


def test_gpu_factor_state_errors(lib):
    from paper_1804_02297_amd import binding
    from paper_1804_02297_amd.binding import LSError, Plan, SparseGpu
    lib_ = binding.load()
    n = 5
    _, rows = _oracle_system(n, 7)
    sp = SparseGpu(n, rows)
    b = I.random_field(1, n, 3)
    st = lib_.ls_sparse_solve_host(sp._h, b.ctypes.data_as(ctypes.c_void_p), 1)
    assert st == -6                                   # a GPU factor has no host solve
    plan = Plan(n, I.wavenumber_for(n), _dev(I.medium_bumps(n, 2)))
    with pytest.raises(LSError) as e:
        plan.factor_gpu()                             # before a stencil fit
    assert e.value.code == -6
    with pytest.raises(LSError) as e:
        SparseGpu(2, np.zeros((8, 3, 27, 3), np.complex128))   # below the smallest grid
    assert e.value.code == -1
