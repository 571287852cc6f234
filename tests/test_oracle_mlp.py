"""Pins of the oracle's stencil-prediction network (a project extension).

* backward() against central finite differences of the loss;
* GELU against x * Phi(x) with SciPy's normal CDF;
* one Adam step moves every parameter by lr * g / (|g| + eps);
* BF16 rounding against torch's bfloat16 cast (round to nearest even);
* target encoding and decoding are inverse to each other.
"""
import math

import numpy as np
import pytest
import scipy.stats

from oracle import mlp
from oracle import stencil as st


def _small_batch(seed, B=4):
    g = np.random.default_rng(seed)
    x = g.standard_normal((B, mlp.D_IN))
    t = 0.1 * g.standard_normal((B, mlp.D_OUT))
    return x, t


def test_backward_matches_finite_differences():
    params = mlp.init_params(3)
    for k in params:
        if k.startswith("b"):
            params[k] = 0.05 * np.random.default_rng(1).standard_normal(params[k].shape)
    x, t = _small_batch(2)
    y, cache = mlp.forward(params, x)
    grads = mlp.backward(params, cache, y, t)
    rng = np.random.default_rng(5)
    eps = 1e-6
    for key in ["W1", "b1", "W2", "b2", "W3", "b3"]:
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in params[key].shape)
            old = params[key][idx]
            params[key][idx] = old + eps
            lp = mlp.loss(mlp.forward(params, x)[0], t)
            params[key][idx] = old - eps
            lm = mlp.loss(mlp.forward(params, x)[0], t)
            params[key][idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - grads[key][idx]) <= 1e-6 * max(1e-8, np.abs(grads[key]).max())


def test_gelu_is_x_times_normal_cdf():
    x = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.gelu(x), x * scipy.stats.norm.cdf(x), rtol=1e-13, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(x), fd, atol=1e-8)


def test_adam_first_step():
    params = {"W": np.array([[1.0, -2.0], [0.5, 0.0]])}
    grads = {"W": np.array([[0.3, -4.0], [1e-3, 2.0]])}
    state = {}
    new = mlp.adam_step({"W": params["W"].copy()}, grads, state, lr=1e-2)
    step = params["W"] - new["W"]
    expect = 1e-2 * grads["W"] / (np.abs(grads["W"]) + 1e-8)
    assert np.allclose(step, expect, rtol=1e-12, atol=0)


def test_bf16_rounding_matches_torch():
    import torch
    g = np.random.default_rng(0)
    a = np.concatenate([g.standard_normal(1000) * 10.0 ** g.integers(-5, 5, 1000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 0.0, -0.0]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.round_bf16(a), ref)


def test_encode_decode_roundtrip():
    g = np.random.default_rng(1)
    base = g.standard_normal((81, 3)) + 1j * g.standard_normal((81, 3))
    base = st.gauge_fix(base)
    other = st.gauge_fix(base + 0.1 * (g.standard_normal((81, 3)) + 1j * g.standard_normal((81, 3))))
    y = mlp.encode_target(other, base)
    assert y.shape == (mlp.D_OUT,)
    back = mlp.decode_output(y, base)
    assert np.abs(back - other).max() <= 1e-13


def test_patch_features_layout():
    n = 6
    m = np.arange(n ** 3).reshape(n, n, n) * (1 + 0.5j) / 100.0
    f = mlp.patch_features(m, [(2, 3, 2), (0, 0, 0)])
    assert f.shape == (2, mlp.D_IN)
    # centre of the patch is entry 62 (= 2*25 + 2*5 + 2)
    assert math.isclose(f[0, 2 * 62], m[2, 3, 2].real / 0.3)
    assert math.isclose(f[0, 2 * 62 + 1], m[2, 3, 2].imag / 0.3)
    # off-grid entries are zero; first in-grid entry of the corner patch is (0,0,0)
    assert f[1, 0] == 0.0 and math.isclose(f[1, 2 * 62], m[0, 0, 0].real / 0.3)


def test_forward_bf16_differs_by_the_activation_rounding_only():
    """forward_bf16 = forward on BF16-rounded weights and inputs, up to the BF16
    rounding of the two hidden activations: each rounded activation moves by at
    most 2^-8 of itself, which propagates to y through |W2| (with GELU's slope,
    at most 1.13) and |W3|.  A first-order bound, with 10 % for the rest."""
    params = mlp.init_params(7)
    g = np.random.default_rng(3)
    for k in ("b1", "b2", "b3"):
        params[k] = 0.05 * g.standard_normal(params[k].shape)
    x = g.standard_normal((16, mlp.D_IN))
    pr = {k: (mlp.round_bf16(v) if k.startswith("W") else v) for k, v in params.items()}
    y, (xx, z1, h1, z2, h2) = mlp.forward(pr, mlp.round_bf16(x))
    yb = mlp.forward_bf16(params, x)
    u = 2.0 ** -8
    dh1 = u * np.abs(h1)
    dh2 = u * np.abs(h2) + 1.13 * dh1 @ np.abs(pr["W2"])
    bound = 1.1 * dh2 @ np.abs(pr["W3"])
    d = np.abs(yb - y)
    assert np.all(d <= bound)
    assert d.max() > 0.0          # the activations are rounded


def test_forward_bf16_is_exact_on_representable_values():
    """With W2 = W3 = 0 only the biases reach y: forward_bf16 == forward exactly."""
    params = mlp.init_params(2)
    params["W2"][:] = 0.0
    params["W3"][:] = 0.0
    params["b3"] = np.linspace(-1.0, 1.0, mlp.D_OUT)
    x = np.random.default_rng(0).standard_normal((3, mlp.D_IN))
    assert np.array_equal(mlp.forward_bf16(params, x), mlp.forward(params, x)[0])
