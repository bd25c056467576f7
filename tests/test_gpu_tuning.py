"""Launch-shape tuning: every option of every choice gives bit-identical
outputs (each output is computed by the same operations in the same order),
and the autotuner leaves a valid choice that reproduces the default run."""
import json
import os

import numpy as np
import pytest
import torch

import synthetic as G
from gpu_util import announce, host, specs
from paper_2106_08817_amd import Plan, _lib

pytestmark = pytest.mark.gpu

N_CHOICES = 6


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


def snapshot(plan):
    torch.cuda.synchronize()
    out = [host(plan.out_cost).copy()]
    for i in range(len(plan.out_grad)):
        out += [host(plan.out_grad[i]).copy(), host(plan.out_image[i]).copy(), host(plan.out_momentum[i]).copy()]
    return out


def assert_same(a, b, what):
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x, y), f"{what}: output {k} differs (max |d| {np.max(np.abs(x - y))})"


def batch(ndim):
    if ndim == 2:
        shapes, T, sig = [(40, 52), (67, 33), (96, 130)], 6, [2.0, 3.3, 5.0]
    else:
        shapes, T, sig = [(12, 17, 20), (9, 33, 14)], 4, [2.0, 1.5]
    pairs = [G.small_pair(s, seed=700 + i, rho=0.4 + 0.1 * i, sigma=sig[i], p0_kind="realistic", lam=0.01)
             for i, s in enumerate(shapes)]
    return pairs, T


@pytest.mark.parametrize("ndim", [2, 3])
def test_every_tuning_option_is_bit_identical(ndim):
    pairs, T = batch(ndim)
    plan = Plan(specs(pairs), T)
    assert plan.tuning == [0] * N_CHOICES
    plan.grad()
    ref = snapshot(plan)
    for k in range(N_CHOICES):
        choice = [0] * N_CHOICES
        choice[k] = 1
        announce(f"ndim {ndim} tuning {choice}")
        plan.tuning = choice
        plan.grad()
        assert_same(snapshot(plan), ref, f"choice {choice}")
    plan.tuning = [1] * N_CHOICES
    plan.grad()
    assert_same(snapshot(plan), ref, "all options 1")


def batch_x4(ndim):
    """Every last extent a multiple of 4 (the matrix-core x-pass runs), with
    ragged row tiles, a ragged 16-column tail and radii up to 30."""
    if ndim == 2:
        shapes, T, sig = [(37, 52), (21, 200), (30, 128)], 5, [2.0, 5.0, 10.0]
    else:
        shapes, T, sig = [(11, 13, 36), (7, 9, 20)], 4, [1.5, 3.0]
    pairs = [G.small_pair(s, seed=740 + i, rho=0.5, sigma=sig[i], p0_kind="realistic", lam=0.01)
             for i, s in enumerate(shapes)]
    return pairs, T


@pytest.mark.parametrize("ndim", [2, 3])
def test_matrix_core_xpass_is_bit_identical(ndim):
    pairs, T = batch_x4(ndim)
    plan = Plan(specs(pairs), T)
    plan.grad()
    ref = snapshot(plan)
    for choice in ([0, 0, 0, 0, 0, 1], [1, 1, 1, 1, 1, 1]):
        announce(f"ndim {ndim} tuning {choice}")
        plan.tuning = choice
        plan.grad()
        assert_same(snapshot(plan), ref, f"choice {choice}")


@pytest.mark.parametrize("ndim", [2, 3])
def test_autotune_picks_valid_choices_and_keeps_results(ndim):
    pairs, T = batch(ndim)
    plan = Plan(specs(pairs), T)
    plan.grad()
    ref = snapshot(plan)
    chosen = plan.autotune()
    assert len(chosen) == N_CHOICES and set(chosen) <= {0, 1}
    assert_same(snapshot(plan), ref, "outputs written by autotune")
    plan.grad()
    assert_same(snapshot(plan), ref, f"after autotune {chosen}")


def test_autotune_cache_miss_hit_and_replacement(tmp_path):
    pairs, T = batch(2)
    path = str(tmp_path / "tune.json")
    arch = torch.cuda.get_device_properties(0).gcnArchName
    plan = Plan(specs(pairs), T)
    plan.grad()
    ref = snapshot(plan)
    chosen, hit = plan.autotune_cached(path)
    assert not hit and len(chosen) == N_CHOICES
    assert_same(snapshot(plan), ref, "outputs written by the cached autotune")
    doc = json.load(open(path))
    key = f"{arch}/{plan.tune_class}"
    assert doc == {"format": "shoot-tune-1", "entries": {key: chosen}}
    # a second plan of the same class takes the stored choices without timing
    other = Plan(specs(pairs), T)
    assert other.tune_class == plan.tune_class
    stored = [1 - c for c in chosen]            # a planted entry proves the read
    json.dump({"format": "shoot-tune-1", "entries": {key: stored, "gfx0/other": [0] * N_CHOICES}}, open(path, "w"))
    got, hit = other.autotune_cached(path)
    assert hit and got == stored and other.tuning == stored
    other.grad()
    assert_same(snapshot(other), ref, "after a cache hit")
    # wrong length or values: a miss, and the entry is replaced; other keys stay
    json.dump({"format": "shoot-tune-1", "entries": {key: [2] * N_CHOICES, "gfx0/other": [1] * N_CHOICES}},
              open(path, "w"))
    got, hit = other.autotune_cached(path)
    assert not hit
    doc = json.load(open(path))
    assert doc["entries"] == {key: got, "gfx0/other": [1] * N_CHOICES}
    # not the format: replaced
    open(path, "w").write("not json")
    got, hit = other.autotune_cached(path)
    assert not hit and json.load(open(path)) == {"format": "shoot-tune-1", "entries": {key: got}}
    # cannot write: SHOOT_E_IO, the choices still set
    bad = str(tmp_path / "missing_dir" / "tune.json")
    with pytest.raises(_lib.ShootError, match="SHOOT_E_IO"):
        other.autotune_cached(bad)
    assert not os.path.exists(bad)
