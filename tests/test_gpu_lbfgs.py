"""Batched L-BFGS (shoot_lbfgs_*) against the oracle's L-BFGS with the same
conventions: cost history and iterates on a ragged batch."""
import numpy as np
import pytest
import torch

import oracle
import synthetic as G
from gpu_util import announce, host, rel, specs
from paper_2106_08817_amd import lbfgs

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


def test_lbfgs_matches_oracle_on_ragged_batch():
    pairs = [G.small_pair((20, 24), seed=31, rho=0.5, sigma=2.0, p0_kind="zero", lam=0.01),
             G.small_pair((26, 19), seed=32, rho=0.3, sigma=1.5, p0_kind="realistic", lam=0.01),
             G.small_pair((33, 28), seed=33, rho=0.8, sigma=2.5, p0_kind="random", lam=0.01)]
    T, iters = 5, 4
    sp = specs(pairs)
    plan, hist, evals = lbfgs(sp, T, iters)
    torch.cuda.synchronize()
    assert all(e >= 1 for e in evals)
    for i, p in enumerate(pairs):
        xO, hO, usedO = oracle.lbfgs(p.source, p.target, p.p0, p.rho, p.sigma, p.lam, T, iters)
        got = [h[i] for h in hist]
        err_c = max(abs(a - b) / abs(b) for a, b in zip(got, hO))
        err_x = rel(host(sp[i].p0), xO)
        announce(f"pair {i}: cost rel {err_c:.2e}, p0 rel {err_x:.2e}, oracle trials {usedO}")
        assert err_c <= 1e-4, (got, hO)
        assert err_x <= 1e-3
        assert got[-1] < got[0]


@pytest.mark.parametrize("c1,trials", [(0.45, 8), (0.999, 2)])
def test_lbfgs_backtracking_and_failed_searches(c1, trials):
    """A demanding sufficient-decrease constant makes the search halve the
    step (and, with two trials, fail and restart); the device follows the
    oracle through both."""
    pairs = [G.small_pair((20, 24), seed=41, rho=0.5, sigma=2.0, p0_kind="realistic", lam=0.01),
             G.small_pair((17, 29), seed=42, rho=0.2, sigma=1.5, p0_kind="zero", lam=0.01)]
    T, iters = 4, 4
    sp = specs(pairs)
    plan, hist, evals = lbfgs(sp, T, iters, c1=c1, trials=trials)
    torch.cuda.synchronize()
    saw = []
    for i, p in enumerate(pairs):
        xO, hO, usedO = oracle.lbfgs(p.source, p.target, p.p0, p.rho, p.sigma, p.lam, T, iters, c1=c1,
                                     trials=trials)
        saw += usedO
        got = [h[i] for h in hist]
        np.testing.assert_allclose(got, hO, rtol=1e-4)
        assert rel(host(sp[i].p0), xO) <= 1e-3
    assert max(saw) > 1, "the case must backtrack"
