"""The Python API over the C ABI: the autograd Function and the batched
convenience call give the plan's own results, which match the oracle."""
import numpy as np
import pytest
import torch

import synthetic as G
from gpu_util import announce, check_grad, dev, host, specs
from paper_2106_08817_amd import Plan, ShootCost, shoot_cost

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


def test_autograd_function_gives_the_adjoint_gradient():
    p = G.small_pair((44, 36), 61, rho=0.4, sigma=2.2, p0_kind="realistic", lam=0.02)
    T = 6
    S, J = dev(p.source), dev(p.target)
    p0 = dev(p.p0).requires_grad_(True)
    H = ShootCost.apply(S, J, p0, p.rho, p.sigma, p.lam, T)
    H.backward()
    plan = Plan(specs([p]), T)
    plan.grad()
    torch.cuda.synchronize()
    assert float(H.detach()) == float(plan.out_cost[0, 0])
    assert np.array_equal(host(p0.grad), host(plan.out_grad[0]))
    check_grad(plan, 0, p, T)
    # the functional form, with an upstream weight
    p0.grad = None
    (3.0 * shoot_cost(S, J, p0, p.rho, p.sigma, p.lam, T)).backward()
    assert np.array_equal(host(p0.grad), host(3.0 * plan.out_grad[0]))


def test_cost_and_grad_returns_the_batch_outputs():
    pairs = [G.small_pair(s, 70 + i, rho=0.3, sigma=1.8) for i, s in enumerate([(30, 41), (52, 28), (36, 36)])]
    plan = Plan(specs(pairs), 4)
    costs, grads = plan.cost_and_grad()
    torch.cuda.synchronize()
    assert costs.shape == (3,) and len(grads) == 3
    assert np.array_equal(host(costs), host(plan.out_cost[:, 0]))
    for i, p in enumerate(pairs):
        assert grads[i].shape == p.source.shape
        check_grad(plan, i, p, 4)
    with pytest.raises(ValueError):
        Plan(specs(pairs), 4, outputs=("image",)).cost_and_grad()


def test_pair_selection_skips_inactive_pairs():
    """Inactive pairs keep the outputs of their last evaluation; active ones
    get exactly what a plan of all pairs gives."""
    shapes = [(40, 52), (33, 29), (61, 47)]
    pairs = [G.small_pair(s, 90 + i, rho=0.5, sigma=2.0, p0_kind="realistic") for i, s in enumerate(shapes)]
    T = 5
    sp = specs(pairs)
    plan = Plan(sp, T)
    plan.grad()
    torch.cuda.synchronize()
    old = [(host(plan.out_grad[i]).copy(), host(plan.out_cost[i]).copy()) for i in range(3)]
    for spec in sp:   # new momenta for every pair
        spec.p0.mul_(0.5)
    plan.set_active([True, False, True])
    plan.grad()
    torch.cuda.synchronize()
    ref = Plan(specs(pairs), T)   # the same pairs (halved p0 from the shared buffers)
    for i, spec in enumerate(sp):
        ref.pairs[i].p0.copy_(spec.p0)
    ref.grad()
    torch.cuda.synchronize()
    for i in (0, 2):
        assert np.array_equal(host(plan.out_grad[i]), host(ref.out_grad[i]))
        assert np.array_equal(host(plan.out_cost[i]), host(ref.out_cost[i]))
    assert np.array_equal(host(plan.out_grad[1]), old[1][0])
    assert np.array_equal(host(plan.out_cost[1]), old[1][1])
    plan.set_active(None)
    plan.grad()
    torch.cuda.synchronize()
    for i in range(3):
        assert np.array_equal(host(plan.out_grad[i]), host(ref.out_grad[i]))


def test_pair_selection_3d_and_descent():
    """3-D pairs in two lanes: an inactive pair's gradient, cost and p0 stay
    as they were through gradient and descent calls; the active ones match a
    plan of them alone, step for step."""
    shapes = [(10, 12, 16), (9, 14, 11), (12, 10, 13)]
    pairs = [G.small_pair(s, 120 + i, rho=0.4, sigma=1.5, p0_kind="realistic") for i, s in enumerate(shapes)]
    T = 4
    sp = specs(pairs)
    plan = Plan(sp, T)
    plan.grad()
    torch.cuda.synchronize()
    g1, c1, p1 = host(plan.out_grad[1]).copy(), host(plan.out_cost[1]).copy(), host(sp[1].p0).copy()
    plan.set_active([True, False, True])
    alone = Plan(specs([pairs[0], pairs[2]]), T)
    for it in range(3):
        plan.descend(0.5, reset=(it == 0))
        alone.descend(0.5, reset=(it == 0))
    torch.cuda.synchronize()
    for i, j in ((0, 0), (2, 1)):
        assert np.array_equal(host(plan.out_grad[i]), host(alone.out_grad[j]))
        assert np.array_equal(host(sp[i].p0), host(alone.pairs[j].p0))
    assert np.array_equal(host(plan.out_grad[1]), g1)
    assert np.array_equal(host(plan.out_cost[1]), c1)
    assert np.array_equal(host(sp[1].p0), p1)
