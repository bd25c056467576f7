"""SHOOT_CHECK_FINITE: clean inputs give the unchecked plan's outputs bit for
bit; a NaN or Inf in a pair's image, target or p0 fails the call with
SHOOT_E_ARG naming that pair, before any output is written."""
import numpy as np
import pytest
import torch

import synthetic as G
from gpu_util import announce, host, specs
from paper_2106_08817_amd import SHOOT_CHECK_FINITE, Plan, ShootError
from paper_2106_08817_amd import _lib

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


def batch():
    shapes = [(40, 52), (67, 33), (30, 45)]
    return [G.small_pair(s, seed=950 + i, rho=0.3, sigma=2.0, p0_kind="realistic", lam=0.01)
            for i, s in enumerate(shapes)], 5


def test_clean_inputs_match_the_unchecked_plan():
    pairs, T = batch()
    sp = specs(pairs)
    a, b = Plan(sp, T), Plan(sp, T, SHOOT_CHECK_FINITE)
    a.grad()
    b.grad()
    torch.cuda.synchronize()
    assert np.array_equal(host(a.out_cost), host(b.out_cost))
    for i in range(len(pairs)):
        assert np.array_equal(host(a.out_grad[i]), host(b.out_grad[i]))


@pytest.mark.parametrize("field,bad,at", [("p0", float("nan"), 1), ("target", float("inf"), 2),
                                          ("source", float("-inf"), 0)])
def test_non_finite_input_fails_before_any_output(field, bad, at):
    pairs, T = batch()
    sp = specs(pairs)
    plan = Plan(sp, T, SHOOT_CHECK_FINITE)
    t = {"p0": sp[at].p0, "target": sp[at].target, "source": sp[at].image}[field]
    t.view(-1)[7] = bad
    plan.out_cost.fill_(-7.0)
    for g in plan.out_grad:
        g.fill_(-7.0)
    torch.cuda.synchronize()
    with pytest.raises(ShootError) as ei:
        plan.grad()
    assert ei.value.status == _lib.SHOOT_E_ARG
    assert f"pair {at}:" in str(ei.value) and "1 non-finite" in str(ei.value)
    torch.cuda.synchronize()
    assert np.all(host(plan.out_cost) == -7.0)
    assert all(np.all(host(g) == -7.0) for g in plan.out_grad)


@pytest.mark.parametrize("ndim", [2, 3])
def test_nan_momentum_without_the_check_propagates(ndim):
    """Without SHOOT_CHECK_FINITE a NaN in one pair's p0 makes that pair's
    cost and gradient NaN; the other pairs of the launch keep the values of a
    plan without the bad pair (a NaN displacement puts the foot at its
    arrival point, inside every staged neighbourhood)."""
    if ndim == 2:
        pairs, T = batch()
    else:
        pairs = [G.small_pair(s, seed=960 + i, rho=0.3, sigma=1.5, p0_kind="realistic", lam=0.01)
                 for i, s in enumerate([(12, 18, 40), (10, 14, 21)])]
        T = 4
    sp = specs(pairs)
    clean = Plan(specs(pairs), T)
    clean.grad()
    sp[0].p0.view(-1)[sp[0].p0.numel() // 2] = float("nan")
    plan = Plan(sp, T)
    plan.grad()
    torch.cuda.synchronize()
    assert np.isnan(host(plan.out_cost[0])[0])
    assert np.isnan(host(plan.out_grad[0])).any()
    for i in range(1, len(pairs)):
        assert np.array_equal(host(plan.out_cost[i]), host(clean.out_cost[i]))
        assert np.array_equal(host(plan.out_grad[i]), host(clean.out_grad[i]))
