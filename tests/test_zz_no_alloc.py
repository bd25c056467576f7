"""GPU tests of shoot_plan_bind_scratch, the entry point for callers that
cannot allocate device memory: plans bound to the library's static scratch
give bit-identical outputs to the same plans bound to a caller workspace (the
same kernels run on the same inputs), over calls in a row with a smaller
input in between and the first plan run again afterwards; plans too large for
the scratch are refused; a descent on a scratch plan must reset after another
scratch plan ran."""
import numpy as np
import pytest
import torch

import synthetic as G
from gpu_util import announce, host, specs
from paper_2106_08817_amd import SHOOT_LANES, SHOOT_NO_GRAPH, Plan, _lib
from paper_2106_08817_amd._lib import ShootError

pytestmark = pytest.mark.gpu

FL = SHOOT_NO_GRAPH | SHOOT_LANES(1)


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


def outputs(plan):
    plan.grad()
    torch.cuda.synchronize()
    g = [host(x).copy() for x in plan.out_grad]
    c = host(plan.out_cost).copy()
    plan.forward()
    torch.cuda.synchronize()
    return g, c, [host(x).copy() for x in plan.out_image], [host(x).copy() for x in plan.out_momentum]


def assert_same(a, b, what):
    for name, xa, xb in zip(("grad", "cost", "image", "momentum"), a, b):
        xa = xa if isinstance(xa, list) else [xa]
        xb = xb if isinstance(xb, list) else [xb]
        for u, v in zip(xa, xb):
            assert np.array_equal(u, v), (what, name, float(np.abs(u - v).max()))


@pytest.mark.parametrize("ndim", [2, 3])
def test_scratch_plan_equals_workspace_plan_on_calls_in_a_row(ndim):
    if ndim == 2:
        big = [G.small_pair(s, 40 + i, rho=0.4, sigma=2.2) for i, s in enumerate([(96, 128), (77, 130), (64, 64)])]
        small = [G.small_pair((33, 47), 51, rho=0.6, sigma=1.7)]
    else:
        big = [G.small_pair(s, 60 + i, rho=0.4, sigma=1.6) for i, s in enumerate([(24, 32, 40), (17, 29, 22)])]
        small = [G.small_pair((12, 14, 18), 71, rho=0.7, sigma=1.3)]
    T = 7
    ref_big = outputs(Plan(specs(big), T, FL))
    scr_big = Plan(specs(big), T, FL, scratch=True)
    assert scr_big.workspace is None
    announce(f"  scratch plan: {scr_big.workspace_bytes} bytes of workspace")
    assert_same(outputs(scr_big), ref_big, "first call")
    assert_same(outputs(scr_big), ref_big, "second call")
    # a smaller input in a second scratch plan, then the first plan again: its
    # descriptors are uploaded again before it runs
    ref_small = outputs(Plan(specs(small), T, FL))
    scr_small = Plan(specs(small), T, FL, scratch=True)
    assert scr_small.workspace_bytes < scr_big.workspace_bytes
    assert_same(outputs(scr_small), ref_small, "smaller input")
    assert_same(outputs(scr_big), ref_big, "first plan after the smaller one")
    scr_small.close()
    scr_big.close()


def test_scratch_refuses_large_plans_and_graph_plans():
    big = [G.small_pair((80, 80, 80), 3, rho=0.5, sigma=2.0)]  # ~100 MB of workspace at T = 15
    with pytest.raises(ShootError) as e:
        Plan(specs(big), 15, FL, scratch=True)
    assert e.value.status == _lib.SHOOT_E_WORKSPACE
    with pytest.raises(ShootError) as e:
        Plan(specs([G.small_pair((32, 40), 4)]), 5, 0, scratch=True)
    assert e.value.status == _lib.SHOOT_E_ARG


def test_scratch_descent_resets_after_another_plan_ran():
    a = [G.small_pair((48, 56), 81, rho=0.5, sigma=2.0)]
    b = [G.small_pair((40, 40), 82, rho=0.5, sigma=2.0)]
    T = 5
    sa = Plan(specs(a), T, FL, scratch=True, outputs=("grad", "cost"))
    ra = Plan(specs(a), T, FL, outputs=("grad", "cost"))
    for plan in (sa, ra):
        plan.descend(0.5, reset=True)
        plan.descend(0.5)
    torch.cuda.synchronize()
    assert np.array_equal(host(sa.pairs[0].p0), host(ra.pairs[0].p0))
    sb = Plan(specs(b), T, FL, scratch=True, outputs=("grad", "cost"))
    sb.grad()
    with pytest.raises(ShootError) as e:
        sa.descend(0.5)
    assert e.value.status == _lib.SHOOT_E_STATE
    sa.descend(0.5, reset=True)
    ra.descend(0.5, reset=True)
    torch.cuda.synchronize()
    assert np.array_equal(host(sa.pairs[0].p0), host(ra.pairs[0].p0))
    assert np.array_equal(host(sa.out_cost), host(ra.out_cost))


def test_scratch_plan_keeps_its_pair_selection_across_other_plans():
    """A pair selection on a scratch plan survives another scratch plan's
    call (whose header overwrote the array): the re-uploaded descriptors
    still skip the inactive pair, whose outputs stay as they were."""
    pairs = [G.small_pair(s, 80 + i, rho=0.5, sigma=1.8) for i, s in enumerate([(40, 52), (33, 29), (48, 36)])]
    other = [G.small_pair((30, 34), 90, rho=0.3, sigma=1.5)]
    T = 5
    sp = specs(pairs)
    a = Plan(sp, T, FL, scratch=True)
    a.grad()
    torch.cuda.synchronize()
    old_g, old_c = host(a.out_grad[1]).copy(), host(a.out_cost[1]).copy()
    for s in sp:
        s.p0.mul_(0.5)
    a.set_active([True, False, True])
    b = Plan(specs(other), T, FL, scratch=True)
    b.grad()                      # the array now holds b's header
    a.grad()                      # a's header, selection included, goes up again
    torch.cuda.synchronize()
    ref = Plan(specs(pairs), T, FL)
    for i, s in enumerate(sp):
        ref.pairs[i].p0.copy_(s.p0)
    ref.grad()
    torch.cuda.synchronize()
    for i in (0, 2):
        assert np.array_equal(host(a.out_grad[i]), host(ref.out_grad[i]))
    assert np.array_equal(host(a.out_grad[1]), old_g)
    assert np.array_equal(host(a.out_cost[1]), old_c)
    a.set_active(None)            # owner now: uploaded at once
    a.grad()
    torch.cuda.synchronize()
    assert np.array_equal(host(a.out_grad[1]), host(ref.out_grad[1]))
