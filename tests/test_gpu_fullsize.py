"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (default plan flags: batched tile lists, sqrt(T) checkpoints,
captured graph). Where the oracle cannot follow the whole workload in seconds,
it checks one step at full size, and the whole run is checked through
properties that hold at any size."""
import numpy as np
import pytest
import torch

import synthetic as G
from gpu_util import announce, check_forward, check_grad, host, rel, run
from paper_2106_08817_amd import SHOOT_FULL_STORE

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


@pytest.fixture(scope="module")
def c3():
    return G.workload("c3")


def test_c3_batch_sampled_pairs_match_oracle(c3):
    """The 64-pair ragged 2-D batch, T = 20, as benchmarked: every cost is
    finite, and sampled pairs (smallest, largest, two others) match the
    oracle's cost and gradient."""
    plan = run(c3.pairs, c3.T, op="grad")
    costs = host(plan.out_cost)
    assert np.all(np.isfinite(costs))
    sizes = [p.size for p in c3.pairs]
    sample = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 17, 42})
    for i in sample:
        announce(f"c3 pair {i} shape {c3.pairs[i].shape}")
        check_grad(plan, i, c3.pairs[i], c3.T)


def test_c2_single_pair_forward_and_gradient():
    w = G.workload("c2")
    p = w.pairs[0]
    plan = run([p], w.T, op="grad")
    check_grad(plan, 0, p, w.T)
    plan.forward()
    torch.cuda.synchronize()
    check_forward(plan, 0, p, w.T)


@pytest.fixture(scope="module")
def c4():
    return G.workload("c4")


def test_c4_one_step_at_full_size_matches_oracle(c4):
    """160x192x160, one step (T = 1) against the oracle: image, momentum,
    cost and gradient."""
    p = c4.pairs[0]
    plan = run([p], 1, op="grad")
    check_grad(plan, 0, p, 1)
    plan.forward()
    torch.cuda.synchronize()
    check_forward(plan, 0, p, 1)


def test_c4_full_run_properties(c4):
    """T = 15: checkpointed and full-store gradients agree, two runs are
    bitwise identical (no atomics on the gather path), and the zero momentum
    reproduces the source exactly."""
    p = c4.pairs[0]
    a = run([p], c4.T, op="grad")
    g1 = host(a.out_grad[0]).copy()
    c1 = host(a.out_cost).copy()
    assert np.all(np.isfinite(g1)) and np.all(np.isfinite(c1))
    a.grad()
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(a.out_grad[0]), g1)
    b = run([p], c4.T, op="grad", flags=SHOOT_FULL_STORE)
    assert rel(host(b.out_grad[0]), g1) <= 1e-6
    z = G.phantom_pair(p.shape, 4, p.rho, p.sigma, p0_kind="zero")
    f = run([z], c4.T, op="forward")
    np.testing.assert_array_equal(f.out_image[0].cpu().numpy(), z.source)


def test_c5_batched_equals_single_pair_plans():
    """Ragged full-size volumes of the 3-D batch in one plan (the first four of
    the sixteen): two sampled pairs equal their own single-pair plans."""
    w = G.workload("c5", n_pairs=4)
    plan = run(w.pairs, w.T, op="grad")
    assert np.all(np.isfinite(host(plan.out_cost)))
    for i in (0, 3):
        announce(f"c5 pair {i} shape {w.pairs[i].shape}")
        single = run([w.pairs[i]], w.T, op="grad")
        assert rel(host(plan.out_grad[i]), host(single.out_grad[0])) <= 1e-6
        np.testing.assert_allclose(host(plan.out_cost[i]), host(single.out_cost[0]), rtol=1e-6)
