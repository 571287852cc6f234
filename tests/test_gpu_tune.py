"""Block right-hand sides and the apply autotuner on the GPU.

Every launch choice (right-hand sides per launch set, pass-3 teams per
workgroup, the row-run length of each strided pass, persistent launches of
the strided passes and of pass 3)
runs the same arithmetic in the same order, so results must be bitwise
identical across choices; the tuned batch apply must also match the oracle
within the FP32 bar.  The tuner's cache file must round-trip.
"""
import json

import numpy as np
import pytest

from oracle import operator as oop
from paper_1804_02297_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _plan(n, max_rhs, cache=None, seed=3):
    from paper_1804_02297_amd.binding import Plan
    m = torch.from_numpy(I.medium_bumps(n, seed)).to("cuda:0")
    return Plan(n, I.wavenumber_for(n), m, max_rhs=max_rhs, tune_cache=cache)


@pytest.mark.parametrize("prec", ["c64", "c128", "mixed"])
def test_launch_choices_bitwise_identical(lib, prec):
    n, B = 50, 4                         # P = 128: teams of one wavefront, 1/2/4 teams allowed
    plan = _plan(n, B)
    assert plan.P == 128
    dt = torch.complex64 if prec == "c64" else torch.complex128
    x = torch.from_numpy(I.random_field(B, n, 11)).to("cuda:0").to(dt)
    ref = plan.apply(x, prec=prec)
    for choice in [(1, 1, 0, 0), (2, 2, 0, 0), (4, 4, 0, 0), (4, 1, 0, 0), (3, 2, 0, 0), (1, 4, 0, 0),
                   (4, 2, 15, 0), (4, 2, 5, 1), (2, 4, 0, 1), (3, 1, 10, 1), (4, 2, 0, 2), (2, 1, 3, 3)]:
        plan.set_tune(prec, *choice)
        y = plan.apply(x, prec=prec)
        assert torch.equal(y, ref), choice
    plan.set_tune(prec, 0, 0)
    plan.close()


@pytest.mark.parametrize("prec", ["c128", "mixed"])
def test_launch_choices_bitwise_identical_p256(lib, prec):
    """P = 256: the paired-lane FP64 pass 3 and the prefetching FP32 one, with
    ordinary and persistent grids, full and half runs."""
    n, B = 97, 2
    plan = _plan(n, B)
    assert plan.P == 256
    x = torch.from_numpy(I.random_field(B, n, 13)).to("cuda:0")
    ref = plan.apply(x, prec=prec)
    for choice in [(1, 1, 0, 0), (2, 2, 0, 1), (2, 1, 15, 1), (1, 2, 6, 0), (2, 2, 0, 2), (1, 1, 9, 3)]:
        plan.set_tune(prec, *choice)
        assert torch.equal(plan.apply(x, prec=prec), ref), choice
    plan.close()


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_launch_choices_bitwise_identical_p384(lib, prec):
    """P = 384: pass 3 with 32-lane jobs (24 active), one or two teams per
    workgroup, ordinary and persistent grids (the default choice's outputs
    are checked against the oracle at P = 384 in test_gpu_apply.py)."""
    n, B = 150, 2
    plan = _plan(n, B)
    assert plan.P == 384
    dt = torch.complex64 if prec == "c64" else torch.complex128
    x = torch.from_numpy(I.random_field(B, n, 14)).to("cuda:0").to(dt)
    ref = plan.apply(x, prec=prec)
    for choice in [(2, 2, 0, 0), (1, 1, 0, 0), (2, 1, 0, 1), (2, 2, 15, 1), (2, 2, 0, 2), (1, 1, 0, 3)]:
        plan.set_tune(prec, *choice)
        assert torch.equal(plan.apply(x, prec=prec), ref), choice
    plan.close()


def test_set_tune_rejects_bad_choices(lib):
    from paper_1804_02297_amd.binding import LSError
    plan = _plan(8, 2)
    for choice in [(3, 0, 0, 0), (-1, 0, 0, 0), (0, 3, 0, 0), (0, 8, 0, 0), (0, 0, 16, 0), (0, 0, -1, 0),
                   (0, 0, 0, 4), (0, 0, 0, -1)]:
        with pytest.raises(LSError):
            plan.set_tune("c64", *choice)
    plan.close()


def test_tune_picks_valid_choice_and_caches(lib, tmp_path):
    cache = str(tmp_path / "tune.json")
    n, B = 50, 8
    plan = _plan(n, B, cache)
    info = plan.tune(B, "c64")
    print("tune", info, flush=True)
    assert info["from_cache"] == 0 and info["n_tried"] >= 4 + 4 + 3
    assert 1 <= info["chunk"] <= B and info["kmul_w"] in (1, 2, 4)
    assert 0 <= info["half_runs"] <= 15 and info["persist"] in (0, 1, 2, 3)
    assert 0 < info["ms_per_rhs"] <= info["ms_default_per_rhs"] * 1.05
    with open(cache) as f:
        entries = json.load(f)
    assert len(entries) == 1 and f"n={n}|P=128|form=0|prec=1|nrhs={B}" in entries[0]["key"]
    assert (entries[0]["half_runs"], entries[0]["persist"]) == (info["half_runs"], info["persist"])
    # the tuned apply still matches the oracle (FP32 bar) on every rhs
    x = I.random_field(B, n, 12)
    y = plan.apply(torch.from_numpy(x).to("cuda:0").to(torch.complex64), prec="c64").cpu().numpy()
    k = I.wavenumber_for(n)
    m = I.medium_bumps(n, 3)
    for r in (0, B - 1):
        ref = oop.apply_fft(n, k, m, x[r:r + 1])[0]
        assert np.abs(y[r] - ref).max() <= 1e-5 * np.abs(ref).max()
    plan.close()
    # a second plan with the same key reads the cache and times nothing
    plan2 = _plan(n, B, cache)
    info2 = plan2.tune(B, "c64")
    assert info2["from_cache"] == 1 and info2["n_tried"] == 0
    keys = ("chunk", "kmul_w", "half_runs", "persist")
    assert [info2[k] for k in keys] == [info[k] for k in keys]
    # another precision adds a second entry
    plan2.tune(B, "mixed")
    with open(cache) as f:
        assert len(json.load(f)) == 2
    plan2.close()


def test_tune_refuses_the_paper_form(lib, tmp_path):
    """The launch choices are the dyadic form's: tuning a plan in the paper's
    form is LS_ESTATE and writes no cache entry."""
    from paper_1804_02297_amd.binding import LSError
    cache = str(tmp_path / "tune.json")
    plan = _plan(12, 4, cache)
    plan.set_form("paper")
    with pytest.raises(LSError) as e:
        plan.tune(4, "c64")
    assert e.value.code == -6
    import os
    assert not os.path.exists(cache)
    plan.set_form("dyadic")
    assert plan.tune(4, "c64")["from_cache"] == 0
    plan.close()
