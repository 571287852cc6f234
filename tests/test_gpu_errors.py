"""Error paths of the C ABI on the GPU: every misuse returns its documented
status and leaves the objects usable (no kernel runs on bad arguments)."""
import ctypes

import numpy as np
import pytest

from paper_1804_02297_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

EINVAL, ESTATE = -1, -6


def _plan(n, max_rhs=1):
    from paper_1804_02297_amd.binding import Plan
    return Plan(n, I.wavenumber_for(n), torch.from_numpy(I.medium_bumps(n, 2)).to("cuda:0"), max_rhs=max_rhs)


def test_network_misuse(lib):
    from paper_1804_02297_amd.binding import LSError, Mlp
    net = Mlp(np.zeros(250324, np.float32))
    with pytest.raises(LSError) as e:
        net.adam_step(1e-3)                          # no backward pass yet
    assert e.value.code == ESTATE
    g = np.random.default_rng(0)
    net.forward_backward(g.standard_normal((4, 250)).astype(np.float32), np.zeros((4, 468), np.float32))
    for lr in (0.0, -1e-3, float("nan")):
        with pytest.raises(LSError) as e:
            net.adam_step(lr)
        assert e.value.code == EINVAL
    net.adam_step(1e-3)                              # now valid
    with pytest.raises(LSError) as e:
        net.train(10, batch=8)                       # no samples
    assert e.value.code == EINVAL
    plan = _plan(8)
    with pytest.raises(LSError) as e:
        net.add_samples(plan, [0])                   # a boundary point
    assert e.value.code == EINVAL
    assert net.num_samples() == 0
    net.add_samples(plan, [np.ravel_multi_index((3, 3, 3), (8, 8, 8))])
    with pytest.raises(LSError) as e:
        net.train(5, batch=8, lr=0.0)
    assert e.value.code == EINVAL
    net.train(5, batch=8)
    small = _plan(3)
    with pytest.raises(LSError) as e:
        small.stencil_fit_learned(net)              # n = 3 has no complement
    assert e.value.code == EINVAL


def test_plan_and_apply_misuse(lib):
    from paper_1804_02297_amd import binding
    from paper_1804_02297_amd.binding import LSError
    lib_ = binding.load()
    plan = _plan(8, max_rhs=2)
    x = torch.zeros((3, 3, 8, 8, 8), dtype=torch.complex128, device="cuda:0")
    y = plan.apply(x, prec="c128")                   # 3 rhs > max_rhs: applied in chunks
    assert torch.equal(y, x)                         # zero input: zero convolution
    st = lib_.ls_apply(plan._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), 1, 7, None)
    assert st == EINVAL                              # unknown precision
    st = lib_.ls_apply(plan._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), 0, 0, None)
    assert st == EINVAL                              # no right-hand side
    with pytest.raises(LSError) as e:
        plan.factor()                                # before a stencil fit
    assert e.value.code == ESTATE
    with pytest.raises(LSError) as e:
        _bad_factor(lib_, plan)                      # unknown factor precision
    assert e.value.code == EINVAL
    with pytest.raises(LSError) as e:
        _plan(193)                                   # above the largest FFT length
    assert e.value.code == EINVAL


def _bad_factor(lib_, plan):
    from paper_1804_02297_amd.binding import _check
    t = ctypes.c_double()
    _check(lib_.ls_factor_prec(plan._h, 9, ctypes.byref(t)), "ls_factor_prec")
