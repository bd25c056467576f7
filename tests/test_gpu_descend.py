"""Device-side gradient descent (shoot_descend) against the oracle's gradient
descent: the same fixed step, halved when a pair's cost rises; cost history
and the p0 reached after a few iterations."""
import numpy as np
import pytest
import torch

import oracle
import synthetic as G
from gpu_util import announce, host, rel, specs
from paper_2106_08817_amd import Plan, ShootError, gradient_descent

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


@pytest.mark.parametrize("p0_kind", ["zero", "realistic"])
def test_descend_matches_oracle_gradient_descent(p0_kind):
    pairs = [G.small_pair((24, 30), seed=900, rho=0.5, sigma=2.0, p0_kind=p0_kind, lam=0.01),
             G.small_pair((37, 21), seed=901, rho=0.2, sigma=1.5, p0_kind=p0_kind, lam=0.01)]
    T, iters, eta = 6, 5, 2.0
    sp = specs(pairs)
    plan, hist = gradient_descent(sp, T, iters, eta)
    torch.cuda.synchronize()
    hist = hist.cpu().numpy().astype(np.float64)
    for i, p in enumerate(pairs):
        pO, hO = oracle.gradient_descent(p.source, p.target, p.p0, p.rho, p.sigma, p.lam, T, iters, eta)
        np.testing.assert_allclose(hist[:, i], hO, rtol=1e-5)
        assert rel(host(sp[i].p0), pO) <= 1e-4


def test_descend_step_halving_and_reset():
    """A step far too large makes the cost rise: the step halves on the
    device; a reset restores eta0."""
    p = G.small_pair((24, 30), seed=905, rho=0.5, sigma=2.0, p0_kind="zero", lam=0.01)
    T, eta = 4, 10.0
    sp = specs([p])
    plan = Plan(sp, T, 0, outputs=("grad", "cost"))
    with pytest.raises(ShootError):
        plan.descend(eta, reset=False)           # the first call after bind must reset
    p0_start = host(sp[0].p0).copy()
    plan.descend(eta, reset=True)
    torch.cuda.synchronize()
    c = [float(plan.out_cost[0, 0])]
    for _ in range(3):
        plan.descend(eta)
        torch.cuda.synchronize()
        c.append(float(plan.out_cost[0, 0]))
    pO, hO = oracle.gradient_descent(p.source, p.target, p0_start, p.rho, p.sigma, p.lam, T, 4, eta)
    np.testing.assert_allclose(c, hO, rtol=1e-4)
    assert any(b > a for a, b in zip(hO, hO[1:])), "the test needs a rising cost"
    assert rel(host(sp[0].p0), pO) <= 1e-4
