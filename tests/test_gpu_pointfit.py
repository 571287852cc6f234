"""GPU parity of the medium-weighted per-point stencil fit (project extension).

Interior points: the span of the GPU's alpha_i equals the span of the oracle's
thin-SVD alpha of M diag(w) (oracle.stencil.fit_point_weighted): projector
difference <= 1e-8 on sampled points; the three eigenvalues of the weighted
Gram equal the oracle's squared singular values to 1e-8 relative.  Boundary
points keep their class stencil.  With m = 0 the fit is the class fit.
"""
import numpy as np
import pytest

from oracle import sparse as osp
from oracle import stencil as ost
from paper_1804_02297_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

LS_FIT_POINT = 1


def _plan(n, m, max_rhs=1):
    from paper_1804_02297_amd.binding import Plan
    return Plan(n, I.wavenumber_for(n), torch.from_numpy(m).to("cuda:0"), max_rhs=max_rhs)


@pytest.mark.parametrize("n,seed", [(6, 0), (10, 1)])
def test_point_fit_matches_oracle(lib, n, seed):
    k = I.wavenumber_for(n)
    m = I.medium_bumps(n, seed)
    print(f"point fit n={n}", flush=True)
    plan = _plan(n, m)
    plan.stencil_fit(LS_FIT_POINT)
    al, ev = plan.point_stencils()
    rng = np.random.default_rng(seed)
    interior = [tuple(rng.integers(1, n - 1, 3)) for _ in range(6)]
    for i0 in interior:
        p = np.ravel_multi_index(i0, (n, n, n))
        oal, obe, osg = ost.fit_point_weighted(m, i0, k, m0=0.1)
        assert np.abs(ost.projector(al[p]) - ost.projector(oal)).max() <= 1e-8, i0
        assert np.allclose(ev[p], osg[:3] ** 2, rtol=1e-8, atol=0), i0
    # boundary points keep their class stencil
    cal, _, _ = plan.class_stencils()
    for i0 in [(0, 2, 3), (n - 1, n - 1, 0), (2, 0, n - 1)]:
        p = np.ravel_multi_index(i0, (n, n, n))
        kap = ost.class_of_point(i0[0] + 1, i0[1] + 1, i0[2] + 1, n)
        assert np.array_equal(al[p], cal[kap])


def test_point_fit_zero_medium_is_class_fit(lib):
    n = 7
    m = np.zeros((n, n, n), complex)
    plan = _plan(n, m)
    plan.stencil_fit(LS_FIT_POINT)
    al, _ = plan.point_stencils()
    cal, _, _ = plan.class_stencils()
    for p in [np.ravel_multi_index((3, 3, 3), (n, n, n)), np.ravel_multi_index((1, 4, 2), (n, n, n))]:
        assert np.abs(ost.projector(al[p]) - ost.projector(cal[13])).max() <= 1e-9


@pytest.mark.parametrize("nrhs", [1, 5, 11])
def test_point_fit_preconditioner_matches_oracle(lib, nrhs):
    """S^-1 Q v with the per-point stencils against the oracle's sparse LU on
    the same stencils, for every rhs (Q v takes one, four or eight rhs per
    thread by batch size; 5 and 11 leave a partial group)."""
    n = 8
    k = I.wavenumber_for(n)
    m = I.medium_bumps(n, 3)
    plan = _plan(n, m, max_rhs=nrhs)
    plan.stencil_fit(LS_FIT_POINT)
    plan.factor()
    al, _ = plan.point_stencils()
    v = I.random_field(nrhs, n, 4)
    z = plan.precond(torch.from_numpy(v).to("cuda:0")).cpu().numpy()
    B13 = ost.local_block(13, n, k)
    cal, cbe, _ = plan.class_stencils()

    def stencil_of(i1, i2, i3, kappa):
        p = (i1 * n + i2) * n + i3
        R = 3 * len(ost.tau_offsets(kappa))
        a = al[p, :R]
        if kappa == 13:
            return a, B13.conj().T @ a
        return a, cbe[kappa, :R]

    S, Q = osp.assemble_pointwise(n, m, stencil_of)
    pre = osp.Preconditioner(S, Q)
    for r in range(nrhs):
        ref = pre(v[r])
        assert np.abs(z[r] - ref).max() <= 1e-9 * np.abs(ref).max(), r
