"""The paper's own 3x4 form of the apply (Section 2) on the GPU against the oracle.

Bar: complex128 to 1e-12 of the output's size, FP32 (complex64 and mixed) to
1e-5, element by element, on grids spanning several FFT sizes and ragged
tails; the right-hand side the same way; a solve of this form reaches the
FP64 residual bar recomputed with the oracle's apply of this form.
"""
import numpy as np
import pytest

from oracle import paper_form as opf
from paper_1804_02297_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _contrast(n, seed):
    g = np.random.default_rng(seed)
    noise = 0.05 * (g.standard_normal((n, n, n)) + 1j * g.standard_normal((n, n, n)))
    return I.medium_bumps(n, seed) + noise


@pytest.mark.parametrize("n", [3, 4, 5, 8, 12, 16, 24])
def test_paper_apply_matches_oracle(lib, n):
    from paper_1804_02297_amd.binding import Plan
    k = I.wavenumber_for(n)
    m = _contrast(n, 40 + n)
    x = I.random_field(2, n, 500 + n)
    print(f"n={n}", flush=True)
    plan = Plan(n, k, _dev(m), max_rhs=2)
    plan.set_form("paper")
    ref = opf.apply_fft_paper(n, k, m, x)
    scale = np.abs(ref).max()
    y = plan.apply(_dev(x), prec="c128").cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-12 * scale
    y = plan.apply(_dev(x), prec="mixed").cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-5 * scale
    y = plan.apply(_dev(x.astype(np.complex64)), prec="c64").cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-5 * scale
    plan.close()


def test_paper_rhs_chunks_and_form_switch(lib):
    from paper_1804_02297_amd.binding import Plan
    n = 10
    k = I.wavenumber_for(n)
    m = _contrast(n, 7)
    Ei = I.plane_waves(n, k, [[1.0, 0, 0], [0, 0.6, 0.8]], [[0, 0, 1.0], [1.0, 0, 0]])
    plan = Plan(n, k, _dev(m), max_rhs=1)
    x = I.random_field(3, n, 9)
    yd = plan.apply(_dev(x)).cpu().numpy()                      # dyadic form
    plan.set_form("paper")
    g = plan.rhs_from_incident(_dev(Ei)).cpu().numpy()
    gref = opf.rhs_from_incident_paper(n, k, m, Ei)
    assert np.abs(g - gref).max() <= 1e-12 * np.abs(gref).max()
    y3 = plan.apply(_dev(x)).cpu().numpy()                      # 3 rhs > max_rhs: chunks of one
    ref = opf.apply_fft_paper(n, k, m, x)
    assert np.abs(y3 - ref).max() <= 1e-12 * np.abs(ref).max()
    plan.set_form("dyadic")
    assert np.array_equal(plan.apply(_dev(x)).cpu().numpy(), yd)


def test_paper_form_solve(lib):
    """FGMRES on the paper's form with the sparsifying preconditioner of the
    class fit; the residual of this form recomputed by the oracle."""
    from paper_1804_02297_amd.binding import Plan
    n = 16
    k = I.wavenumber_for(n)
    m = I.medium_bumps(n, 1)
    Ei = I.paper_incident(n, k)
    plan = Plan(n, k, _dev(m), max_rhs=1)
    plan.stencil_fit()
    plan.factor_gpu("c128")
    plan.set_form("paper")
    g = plan.rhs_from_incident(_dev(Ei))
    x, info, st = plan.solve(g, tol=1e-8, restart=30)
    assert st == 0, info
    gh = opf.rhs_from_incident_paper(n, k, m, Ei)
    r = gh - opf.apply_fft_paper(n, k, m, x.cpu().numpy())
    rr = np.linalg.norm(r) / np.linalg.norm(gh)
    print("paper form: iterations", info[0]["iters"], "oracle residual", rr, flush=True)
    assert rr <= 1e-8
