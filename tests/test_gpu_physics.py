"""The static limit through the GPU path (plan, class fit, GPU factor, FGMRES).

The scattered field solved on the GPU plus the incident field must give the
closed-form interior field of a small homogeneous scatterer: 3 E0 / (eps + 2)
in a sphere (3-D dyadic form with its self term) and 2 E0 / (eps + 1) in a
circular cylinder (the 2-D paper form), eps = 1 - m; the same bounds as the
oracle's pins of these limits.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

K_STATIC = 0.05


def _ball(n, R=0.3, dim=3):
    h = 1.0 / (n + 1)
    x = (np.arange(n) + 1) * h
    X = np.meshgrid(*([x] * dim), indexing="ij")
    r = np.sqrt(sum((Xd - .5) ** 2 for Xd in X))
    return X[0], r, h


@pytest.mark.parametrize("mval", [-0.5, 0.4])
def test_gpu_sphere_static_limit(lib, mval):
    from paper_1804_02297_amd.binding import Plan
    n, R = 16, 0.3
    X1, r, h = _ball(n, R, 3)
    m = np.where(r < R, mval, 0.0).astype(np.complex128)
    Ei = np.zeros((1, 3, n, n, n), np.complex128)
    Ei[0, 2] = np.exp(1j * K_STATIC * X1)
    print(f"sphere n={n} m={mval}", flush=True)
    plan = Plan(n, K_STATIC, torch.from_numpy(m).to("cuda:0"), max_rhs=1)
    Eid = torch.from_numpy(Ei).to("cuda:0")
    g = plan.rhs_from_incident(Eid)
    plan.stencil_fit()
    plan.factor_gpu("c128")
    x, info, st = plan.solve(g, tol=1e-10, restart=30, maxit=300)
    assert st == 0, info
    E = (Eid + x).cpu().numpy()[0]
    deep = r < R - 1.5 * h
    mean = (E[2] / Ei[0, 2])[deep].real.mean()
    exact = 3.0 / (3.0 - mval)
    print(f"  iterations {info[0]['iters']}, mean E_z/E0 {mean:.5f}, closed form {exact:.5f}", flush=True)
    assert abs(mean / exact - 1) < 0.01
    assert np.abs(E[0][deep]).max() < 0.02
    plan.close()


@pytest.mark.parametrize("mval", [-0.5, 0.4])
def test_gpu_cylinder_static_limit(lib, mval):
    from paper_1804_02297_amd.binding import Plan2
    n, R = 80, 0.3
    X1, r, h = _ball(n, R, 2)
    m = np.where(r < R, mval, 0.0).astype(np.complex128)
    Ei = np.zeros((1, 2, n, n), np.complex128)
    Ei[0, 1] = np.exp(1j * K_STATIC * X1)
    print(f"cylinder n={n} m={mval}", flush=True)
    plan = Plan2(n, K_STATIC, torch.from_numpy(m).to("cuda:0"), max_rhs=1)
    Eid = torch.from_numpy(Ei).to("cuda:0")
    g = plan.rhs_from_incident(Eid)
    plan.stencil_fit()
    plan.factor_gpu("c128")
    x, info, st = plan.solve(g, tol=1e-10, restart=30, maxit=300)
    assert st == 0, info
    E = (Eid + x).cpu().numpy()[0]
    deep = r < R - 2.5 * h
    mean = (E[1] / Ei[0, 1])[deep].real.mean()
    exact = 2.0 / (2.0 - mval)
    print(f"  iterations {info[0]['iters']}, mean E_2/E0 {mean:.5f}, closed form {exact:.5f}", flush=True)
    assert abs(mean / exact - 1) < 0.02
    assert np.abs(E[0][deep]).max() < 0.03
    plan.close()
