"""The 2-D variant on the GPU against the oracle (paper form with the 2-D
Helmholtz kernel, two components).

Bar: complex128 to 1e-12 of the output's size, FP32 (complex64 and mixed) to
2e-5 (FFT rounding of length-P transforms, P <= 1944: a few 1e-7 per
transform, with the symbol's spread of magnitudes), element by element, on
grids spanning radix-4/2/3 lengths and ragged row and column blocks.
"""
import numpy as np
import pytest

from oracle import two_d as o2
from paper_1804_02297_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("n", [3, 4, 5, 9, 12, 17, 25, 40, 61])
def test_apply_matches_oracle(lib, n):
    from paper_1804_02297_amd.binding import Plan2
    k = I.paper_wavenumber(n)
    m = I.medium2_random_complex(n, 30 + n, scale=0.2)
    x = I.random_field2(3, n, 300 + n)
    print(f"n={n}", flush=True)
    plan = Plan2(n, k, _dev(m), max_rhs=2)
    assert plan.P == 2 * n if n in (3, 4, 9, 12) else plan.P >= 2 * n - 1
    ref = o2.apply_fft2(n, k, m, x)
    scale = np.abs(ref).max()
    y = plan.apply(_dev(x), prec="c128").cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-12 * scale
    y = plan.apply(_dev(x), prec="mixed").cpu().numpy()
    assert np.abs(y - ref).max() <= 2e-5 * scale
    y = plan.apply(_dev(x.astype(np.complex64)), prec="c64").cpu().numpy()
    assert np.abs(y - ref).max() <= 2e-5 * scale
    plan.close()


@pytest.mark.parametrize("n", [119, 239, 479])
def test_apply_paper_lengths(lib, n):
    """The kernels compiled for the paper's FFT lengths (P = 256, 486, 972 at
    n = 119, 239, 479), element by element against the oracle's FFT apply
    (itself pinned to the double sum), two rhs, all three precisions."""
    from paper_1804_02297_amd.binding import Plan2
    k = I.paper_wavenumber(n)
    m = I.medium2_perturbed_square(n, n)
    x = I.random_field2(2, n, 7 + n)
    print(f"n={n}", flush=True)
    plan = Plan2(n, k, _dev(m), max_rhs=2)
    assert plan.P == {119: 256, 239: 486, 479: 972}[n]
    ref = o2.apply_fft2(n, k, m, x)
    scale = np.abs(ref).max()
    assert np.abs(plan.apply(_dev(x)).cpu().numpy() - ref).max() <= 1e-12 * scale
    assert np.abs(plan.apply(_dev(x), prec="mixed").cpu().numpy() - ref).max() <= 2e-5 * scale
    y = plan.apply(_dev(x.astype(np.complex64)), prec="c64").cpu().numpy()
    assert np.abs(y - ref).max() <= 2e-5 * scale
    plan.close()


def test_rhs_and_dense_definition(lib):
    """The right-hand side, and the apply against the literal double sum."""
    from paper_1804_02297_amd.binding import Plan2
    n = 7
    k = I.paper_wavenumber(n)
    m = I.medium2_lens(n)
    Ei = I.paper_incident2(n, k)
    plan = Plan2(n, k, _dev(m))
    g = plan.rhs_from_incident(_dev(Ei)).cpu().numpy()
    gref = o2.rhs2(n, k, m, Ei)
    assert np.abs(g - gref).max() <= 1e-12 * np.abs(gref).max()
    x = I.random_field2(1, n, 5)
    y = plan.apply(_dev(x)).cpu().numpy()[0]
    ref = o2.apply_dense2(n, k, m, x[0])
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()


def test_full_size_sampled(lib):
    """The paper's largest 2-D grid (n = 959, P = 1944): sampled outputs of the
    complex128 apply against the oracle's double sum, one output at a time."""
    from paper_1804_02297_amd.binding import Plan2
    n = 959
    k = I.paper_wavenumber(n)
    m = I.medium2_perturbed_square(n, 4)
    x = I.random_field2(2, n, 77)
    plan = Plan2(n, k, _dev(m), max_rhs=2)
    assert plan.P == 1944
    y = plan.apply(_dev(x)).cpu().numpy()
    yf = plan.apply(_dev(x), prec="mixed").cpu().numpy()
    p = o2.gradient_p2(n, m)
    u = np.concatenate([m[None] * x[:, :1], m[None] * x[:, 1:2], (p[0] * x[:, 0] + p[1] * x[:, 1])[:, None]], axis=1)
    s = np.arange(n)
    rng = np.random.default_rng(3)
    for _ in range(6):
        b, d, i1, i2 = rng.integers(2), rng.integers(2), rng.integers(n), rng.integers(n)
        r = np.stack(np.meshgrid(i1 - s, i2 - s, indexing="ij"), axis=-1)
        W = o2.weights_at(r, n, k)
        ref = x[b, d, i1, i2] + k * k * np.sum(W[0] * u[b, d]) + np.sum(W[1 + d] * u[b, 2])
        assert abs(y[b, d, i1, i2] - ref) <= 1e-11 * abs(ref), (b, d, i1, i2)
        assert abs(yf[b, d, i1, i2] - ref) <= 1e-4 * abs(ref), (b, d, i1, i2)


def _projector(a):
    return a @ a.conj().T


@pytest.mark.parametrize("n", [6, 13, 32])
def test_class_stencils_match_oracle(lib, n):
    """The two-dimensional subspace of alpha (alpha is fixed up to a 2 x 2
    unitary factor, the two smallest eigenvalues being a near-degenerate
    pair) and the Ky Fan value: projectors to 1e-9, eigenvalues to 1e-9 of
    the largest."""
    from paper_1804_02297_amd.binding import Plan2
    k = I.paper_wavenumber(n)
    m = I.medium2_lens(n)
    plan = Plan2(n, k, _dev(m))
    plan.stencil_fit()
    a, b, e = plan.stencils()
    print(f"n={n}", flush=True)
    for kappa in range(9):
        ao, bo, so = o2.fit_class2(kappa, n, k)
        D = ao.shape[0]
        assert np.abs(_projector(a[kappa, :D]) - _projector(ao)).max() <= 1e-9
        assert np.abs(e[kappa, :2] - np.sort(so ** 2)[:2]).max() <= 1e-9 * so.max() ** 2
        # beta = B^H alpha for the returned alpha
        tau = o2.tau_offsets2(kappa)
        B = o2.coupling_block2(tau, tau, n, k)
        assert np.abs(b[kappa, :3 * len(tau)] - B.conj().T @ a[kappa, :D]).max() <= 1e-10 * np.abs(B).max()


@pytest.mark.parametrize("n,prec,tol,where", [(12, "c128", 1e-10, "host"), (27, "c128", 1e-10, "host"),
                                              (27, "c64", 2e-4, "host"), (12, "c128", 1e-10, "gpu"),
                                              (27, "c128", 1e-10, "gpu"), (61, "c128", 1e-10, "gpu"),
                                              (27, "c64", 2e-4, "gpu")])
def test_preconditioner_matches_oracle(lib, n, prec, tol, where):
    """z = S^-1 Q v is unique (independent of the unitary freedom in alpha):
    element by element against the oracle's rows factored by SuperLU, with
    S factored on host cores or on the GPU."""
    import oracle.sparse as osp
    from paper_1804_02297_amd.binding import Plan2
    k = I.paper_wavenumber(n)
    m = I.medium2_perturbed_square(n, 2)
    plan = Plan2(n, k, _dev(m), max_rhs=2)
    plan.stencil_fit()
    print(f"n={n} {prec} {where}", flush=True)
    if where == "gpu":
        plan.factor_gpu(prec)
    else:
        plan.factor(prec)
    v = I.random_field2(2, n, 11)
    z = plan.precond(_dev(v)).cpu().numpy()
    al, be, _ = o2.fit_all_classes2(n, k)
    S, Q = o2.assemble2(n, m, al, be)
    P = osp.Preconditioner(S, Q)
    for r in range(2):
        ref = P(v[r])
        assert np.abs(z[r] - ref).max() <= tol * np.abs(ref).max(), r


def test_solve_paper_square(lib):
    """FGMRES with the sparsifying preconditioner on the analogue of the
    paper's 2-D square obstacle at six points per wavelength; the residual
    recomputed with the oracle's apply; the iteration count of the oracle's
    own preconditioned GMRES (4 at this size)."""
    from paper_1804_02297_amd.binding import Plan2
    n = 39
    k = I.paper_wavenumber(n)
    m = I.medium2_square(n)
    Ei = I.paper_incident2(n, k)
    plan = Plan2(n, k, _dev(m))
    plan.stencil_fit()
    plan.factor("c128")
    g = plan.rhs_from_incident(_dev(Ei))
    x, info, st = plan.solve(g, tol=1e-6, restart=20)
    assert st == 0, info
    gh = o2.rhs2(n, k, m, Ei[0])
    r = gh - o2.apply_fft2(n, k, m, x.cpu().numpy()[0])
    rr = np.linalg.norm(r) / np.linalg.norm(gh)
    print("2-D square: iterations", info[0]["iters"], "oracle residual", rr, flush=True)
    assert rr <= 1e-6 and info[0]["iters"] <= 5
    x2, info2, st2 = plan.solve(g, tol=1e-10, restart=20, prec="mixed")
    assert st2 == 0
    r = gh - o2.apply_fft2(n, k, m, x2.cpu().numpy()[0])
    assert np.linalg.norm(r) / np.linalg.norm(gh) <= 1e-10
    # the same solve with the factor in HBM: the same iteration count
    plan.factor_gpu("c128")
    x3, info3, st3 = plan.solve(g, tol=1e-6, restart=20)
    assert st3 == 0 and info3[0]["iters"] == info[0]["iters"]
    r = gh - o2.apply_fft2(n, k, m, x3.cpu().numpy()[0])
    assert np.linalg.norm(r) / np.linalg.norm(gh) <= 1e-6


def test_errors(lib):
    from paper_1804_02297_amd.binding import LSError, Plan2
    n = 3
    plan = Plan2(n, 5.0, _dev(I.medium2_lens(n)))
    with pytest.raises(LSError):
        plan.stencil_fit()                        # n = 3: the interior complement is empty
    n = 8
    plan = Plan2(n, 5.0, _dev(I.medium2_lens(n)))
    g = _dev(I.random_field2(1, n, 1))
    with pytest.raises(LSError):
        plan.factor()                             # before the fit
    with pytest.raises(LSError):
        plan.solve(g)                             # before the factor
    with pytest.raises(ValueError):
        plan.apply(_dev(I.random_field2(1, n + 1, 1)))


def test_size_limits(lib):
    """n = 972 is the largest grid (P = 1944 keeps the FP64 transforms in
    64 KiB of LDS); n = 973 is refused before any device work."""
    from paper_1804_02297_amd.binding import LSError, Plan2
    with pytest.raises(LSError):
        Plan2(973, 5.0, torch.zeros((973, 973), dtype=torch.complex128, device="cuda:0"))


def test_paper_2d_claim(lib):
    """The paper's 2-D claim (fewer than ten GMRES(20) iterations to 1e-6 at
    six points per wavelength) on the analogues of its three 2-D media at its
    smallest 2-D grid, n = 119, with the residual recomputed by the oracle."""
    import json
    import os
    from paper_1804_02297_amd.binding import Plan2
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tables_2d.json")))
    n = 119
    k = I.paper_wavenumber(n)
    Ei = I.paper_incident2(n, k)
    sym = o2.symbol2(n, k)
    for name, gen in I.PAPER_MEDIA_2D.items():
        m = gen(n)
        plan = Plan2(n, k, _dev(m))
        plan.stencil_fit()
        plan.factor("c128")
        g = plan.rhs_from_incident(_dev(Ei))
        x, info, st = plan.solve(g, tol=1e-6, restart=20)
        gh = o2.rhs2(n, k, m, Ei[0], sym)
        r = gh - o2.apply_fft2(n, k, m, x.cpu().numpy()[0], sym)
        rr = np.linalg.norm(r) / np.linalg.norm(gh)
        print(name, "iterations", info[0]["iters"], "oracle residual", rr, flush=True)
        assert st == 0 and rr <= 1.01e-6
        assert info[0]["iters"] < gold["claim_max_iters"]
        plan.close()
