"""Launch-shape tuning: every option of every choice gives bit-identical
outputs (each output is computed by the same operations in the same order),
and the autotuner leaves a valid choice that reproduces the default run."""
import numpy as np
import pytest
import torch

import synthetic as G
from gpu_util import announce, host, specs
from paper_2106_08817_amd import Plan

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
