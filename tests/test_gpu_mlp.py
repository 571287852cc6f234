"""GPU parity of the stencil network (project extension) and the learned fit.

* forward and backward against the oracle's FP64 network with the same BF16
  weights and inputs: outputs within 2e-2 of their maximum, every gradient
  block within 2e-2 of its norm (the GPU rounds activations and gradients to
  BF16 before each product; FP32 accumulation);
* one Adam step against the oracle's Adam on the same gradient;
* training samples (features, gauge-fixed targets) against the oracle's
  patch features and encode_target of the exact per-point fit;
* training lowers the loss; checkpoints round-trip;
* the learned fit falls back to the exact fit when the network carries no
  information (zero or random weights), and with a trained network it solves
  to the FP64 residual bar.
"""
import time

import numpy as np
import pytest

from oracle import mlp as omlp
from oracle import operator as oop
from oracle import stencil as ost
from paper_1804_02297_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _plan(n, m, max_rhs=1):
    from paper_1804_02297_amd.binding import Plan
    return Plan(n, I.wavenumber_for(n), torch.from_numpy(m).to("cuda:0"), max_rhs=max_rhs)


def _params(seed, bias_scale=0.05):
    p = omlp.init_params(seed)
    g = np.random.default_rng(seed + 1)
    for k in ("b1", "b2", "b3"):
        p[k] = bias_scale * g.standard_normal(p[k].shape)
    return p


def test_forward_backward_matches_oracle(lib):
    from paper_1804_02297_amd.binding import Mlp
    p = _params(3)
    flat = Mlp.flat(p)
    net = Mlp(flat)
    g = np.random.default_rng(4)
    B = 96
    x = g.standard_normal((B, 250)).astype(np.float32)
    t = (0.1 * g.standard_normal((B, 468))).astype(np.float32)
    y, grad, loss = net.forward_backward(x, t)
    # oracle with BF16-rounded weights (biases stay FP32) and BF16-rounded inputs
    po = Mlp.unflat(flat.astype(np.float64))
    for k in ("W1", "W2", "W3"):
        po[k] = omlp.round_bf16(po[k])
    xo = omlp.round_bf16(x.astype(np.float64))
    yo, cache = omlp.forward(po, xo)
    go = omlp.backward(po, cache, yo, t.astype(np.float64))
    assert np.abs(y - yo).max() <= 2e-2 * np.abs(yo).max()
    assert abs(loss - omlp.loss(yo, t)) <= 2e-2 * omlp.loss(yo, t)
    gg = Mlp.unflat(grad)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        err = np.linalg.norm(gg[k] - go[k]) / np.linalg.norm(go[k])
        assert err <= 2e-2, (k, err)


def test_inference_matches_oracle_and_training_forward(lib):
    """The fused inference (the learned fit's network evaluation) over a
    ragged number of rows (1000 = 31 tiles of 32 + 8) against the oracle's
    forward with BF16 operands and against the training forward pass: both
    round the same BF16 operands and differ only in the order of the FP32
    sums (bound 2^-10 of the largest output, the BF16 rounding of one
    activation)."""
    from paper_1804_02297_amd.binding import Mlp
    p = _params(7)
    flat = Mlp.flat(p)
    net = Mlp(flat)
    g = np.random.default_rng(8)
    B = 1000
    x = g.standard_normal((B, 250)).astype(np.float32)
    y = net.forward(x)
    yt, _, _ = net.forward_backward(x, np.zeros((B, 468), np.float32))
    yo = omlp.forward_bf16(Mlp.unflat(flat.astype(np.float64)), x.astype(np.float64))
    scale = np.abs(yo).max()
    assert np.abs(y - yo).max() <= 2.0 ** -10 * scale
    assert np.abs(y - yt).max() <= 2.0 ** -10 * scale
    # the same rows alone give the same outputs (the tiling does not matter)
    assert np.array_equal(net.forward(x[992:]), y[992:])


def test_adam_step_matches_oracle(lib):
    from paper_1804_02297_amd.binding import Mlp
    p = _params(5)
    net = Mlp(Mlp.flat(p))
    g = np.random.default_rng(6)
    x = g.standard_normal((32, 250)).astype(np.float32)
    t = g.standard_normal((32, 468)).astype(np.float32)
    p0 = net.params().astype(np.float64)
    _, grad, _ = net.forward_backward(x, t)
    net.adam_step(1e-3)
    p1 = net.params().astype(np.float64)
    ref = omlp.adam_step(Mlp.unflat(p0), Mlp.unflat(grad.astype(np.float64)), {}, lr=1e-3)
    ref = Mlp.flat(ref).astype(np.float64)
    assert np.abs(p1 - ref).max() <= 1e-6


def test_samples_match_oracle(lib):
    from paper_1804_02297_amd.binding import Mlp
    n = 8
    k = I.wavenumber_for(n)
    m = I.medium_bumps(n, 7)
    plan = _plan(n, m)
    net = Mlp(Mlp.flat(_params(1)))
    pts0 = [(3, 3, 3), (1, 4, 6), (5, 2, 3), (6, 6, 1)]
    net.add_samples(plan, [np.ravel_multi_index(q, (n, n, n)) for q in pts0])
    xs, ts = net.samples()
    assert xs.shape == (4, 256)
    cal = ost.gauge_fix(ost.fit_class(13, n, k)[0])
    feats = omlp.round_bf16(omlp.patch_features(m, pts0))
    assert np.array_equal(xs[:, :250], feats.astype(np.float32))
    assert not xs[:, 250:].any()
    for q, i0 in enumerate(pts0):
        al, _, _ = ost.fit_point_weighted(m, i0, k, m0=0.1)
        assert ost.gauge_condition(al) <= 1e6        # all four are kept
        ref = omlp.encode_target(ost.gauge_fix(al), cal)
        assert np.abs(ts[q] - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max()), i0


def test_training_lowers_loss_and_checkpoint_roundtrip(lib, tmp_path):
    from paper_1804_02297_amd.binding import Mlp
    net = Mlp(Mlp.flat(_params(2)))
    for seed in (10, 11):
        n = 10
        plan = _plan(n, I.medium_bumps(n, seed))
        rng = np.random.default_rng(seed)
        pts = rng.choice([(a * n + b) * n + c for a in range(1, n - 1) for b in range(1, n - 1)
                          for c in range(1, n - 1)], 200, replace=False)
        net.add_samples(plan, pts)
    assert net.num_samples() == 400
    loss = net.train(300, batch=128, lr=1e-3, seed=0)
    print("loss first/last", loss[:3], loss[-3:], flush=True)
    assert np.mean(loss[-20:]) < 0.5 * np.mean(loss[:20])
    path = str(tmp_path / "w.lsmlp")
    net.save(path)
    net2 = Mlp(path=path)
    assert np.array_equal(net2.params(), net.params())


def test_learned_fit_falls_back_without_information(lib):
    from paper_1804_02297_amd.binding import Mlp
    n = 8
    m = I.medium_bumps(n, 3)
    n_int = (n - 2) ** 3
    plan = _plan(n, m)
    plan.stencil_fit(1)
    exact, _ = plan.point_stencils()
    zero = Mlp(np.zeros(250324, np.float32))
    assert plan.stencil_fit_learned(zero) == n_int        # predicts the class stencil: not better
    al, _ = plan.point_stencils()
    p = np.ravel_multi_index((3, 4, 3), (n, n, n))
    assert np.abs(ost.projector(al[p]) - ost.projector(exact[p])).max() <= 1e-9
    noisy = Mlp((np.random.default_rng(0).standard_normal(250324) * 3.0).astype(np.float32))
    assert plan.stencil_fit_learned(noisy) == n_int


def test_learned_path_solves(lib):
    """Train on a few media, fit an unseen one, FGMRES to 1e-8 (oracle residual)."""
    from paper_1804_02297_amd.binding import Mlp
    n = 12
    k = I.wavenumber_for(n)
    net = Mlp(Mlp.flat(_params(8)))
    interior = [(a * n + b) * n + c for a in range(1, n - 1) for b in range(1, n - 1) for c in range(1, n - 1)]
    for seed in range(20, 24):
        plan = _plan(n, I.medium_bumps(n, seed))
        net.add_samples(plan, interior)
    net.train(600, batch=512, lr=1e-3, seed=1)
    m = I.medium_bumps(n, 99)
    plan = _plan(n, m)
    Ei = I.plane_waves(n, k, [[1.0, 0, 0]], [[0, 0, 1.0]])
    g = plan.rhs_from_incident(torch.from_numpy(Ei).to("cuda:0"))
    its, secs = {}, {}
    for name in ("class", "point", "learned"):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if name == "learned":
            nfb = plan.stencil_fit_learned(net)
        else:
            plan.stencil_fit(0 if name == "class" else 1)
        torch.cuda.synchronize()
        secs[name] = time.perf_counter() - t0
        plan.factor()
        x, info, st = plan.solve(g, tol=1e-8)
        assert st == 0
        r = g.cpu().numpy() - oop.apply_fft(n, k, m, x.cpu().numpy())
        rel = np.linalg.norm(r) / np.linalg.norm(g.cpu().numpy())
        assert rel <= 1e-8
        its[name] = info[0]["iters"]
    print("iterations", its, "fit seconds", secs, "fallback", nfb, "of", len(interior), flush=True)
    assert nfb <= len(interior) // 2
    assert its["learned"] <= its["class"]
