"""Deformation map psi_T of shoot_forward (out_deformation) against the
oracle: ragged 2-D and 3-D batches, a full-size 2-D pair, and the identity at
zero momentum on full-size batch shapes."""
import numpy as np
import pytest
import torch

import oracle
import synthetic as G
from gpu_util import announce, host, rel, specs
from paper_2106_08817_amd import Plan

pytestmark = pytest.mark.gpu
DEF_TOL = 1e-5


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


def shoot_def(pairs, T):
    plan = Plan(specs(pairs), T, 0, outputs=("image", "momentum", "deformation"))
    plan.forward()
    torch.cuda.synchronize()
    return plan


@pytest.mark.parametrize("ndim", [2, 3])
def test_deformation_matches_oracle_on_ragged_batch(ndim):
    if ndim == 2:
        shapes, T, sig = [(40, 52), (67, 33), (96, 130)], 8, [2.0, 3.3, 5.0]
    else:
        shapes, T, sig = [(12, 17, 20), (9, 33, 14)], 5, [2.0, 1.5]
    pairs = [G.small_pair(s, seed=800 + i, rho=0.3 + 0.2 * i, sigma=sig[i], p0_kind="realistic", lam=0.01)
             for i, s in enumerate(shapes)]
    plan = shoot_def(pairs, T)
    for i, p in enumerate(pairs):
        want = oracle.deformation(p.source, p.p0, p.rho, p.sigma, T)
        got = host(plan.out_deformation[i])
        assert got.shape == want.shape
        e = rel(got, want)
        assert e <= DEF_TOL, f"pair {i} {p.shape}: psi rel {e:.2e}"
        # the image output of the same call is unchanged by the extra output
        tr = oracle.shoot(p.source, p.p0, p.rho, p.sigma, T)
        assert rel(host(plan.out_image[i]), tr.I[-1]) <= 1e-5


def test_deformation_full_size_pair():
    w = G.workload("c2")
    p = w.pairs[0]
    plan = shoot_def([p], w.T)
    want = oracle.deformation(p.source, p.p0, p.rho, p.sigma, w.T)
    assert rel(host(plan.out_deformation[0]), want) <= DEF_TOL


def test_zero_momentum_gives_identity_on_batch_shapes():
    w = G.workload("c3", p0_kind="zero", n_pairs=6)
    plan = shoot_def(w.pairs, w.T)
    for i, p in enumerate(w.pairs):
        np.testing.assert_array_equal(host(plan.out_deformation[i]), oracle.grid_coords(p.shape))
