"""GPU parity of every code path of the adjoint advection against the oracle.

The transpose of the interpolation (adjoint of the semi-Lagrangian step,
Methods) runs in one of three ways per pair and step, chosen from the largest
displacement D = max |dt v| of that step that the forward pass recorded:

* 2-D, D < 1 px: gather over the fixed 3x3 stencil;
* 2-D, 1 <= D < 2 px: gather over the general (2H+1)^2 stencil, H = floor(D)+1;
* 2-D, D >= 2 px, and 3-D, D >= 3 voxels: scatter through global atomics
  (also forced by SHOOT_FORCE_GLOBAL_SCATTER);
* 3-D, D < 1 voxel: gather over the fixed 3x3x3 stencil;
* 3-D, 1 <= D < 2 voxels: scatter through LDS atomics into a box over the
  tile grown by 2 (foot corners from the staged fields), flushed with one
  global atomic per touched cell;
* 3-D, 2 <= D < 3 voxels: the same into a box over the tile grown by 3
  (foot corners from global memory).

Each test builds inputs whose steps take the intended path, asserts that from
the oracle's own trajectory (every step's D), and compares cost, gradient
(relative L2 and per element), final image and momentum with the oracle.
rho is small (0.003) so that momenta large enough to move feet by several
pixels per step keep the trajectory bounded (the residual term rho z would
otherwise build steep intensities that feed the velocity back), while the
intensity-residual path of the adjoint stays live."""
import numpy as np
import pytest
import torch

import oracle
import synthetic as G
from gpu_util import announce, check_forward, check_grad, run
from paper_2106_08817_amd import SHOOT_FORCE_GLOBAL_SCATTER

pytestmark = pytest.mark.gpu

RHO = 0.003


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


def steps_D(p, T):
    """Largest |dt v| of every step of the oracle's trajectory."""
    tr = oracle.shoot(p.source, p.p0, p.rho, p.sigma, T)
    return [max(float(np.abs(va).max()) / T for va in vt) for vt in tr.v]


def pair(shape, sigma, amp, seed=123):
    return G.small_pair(shape, seed, rho=RHO, sigma=sigma, amplitude=amp)


def check_all(pairs, T, flags=0):
    plan = run(pairs, T, op="grad", flags=flags)
    for i, p in enumerate(pairs):
        check_grad(plan, i, p, T)
    plan.forward()
    torch.cuda.synchronize()
    for i, p in enumerate(pairs):
        check_forward(plan, i, p, T)


def test_2d_general_gather_every_step():
    p = pair((48, 56), 2.0, 120.0)
    T = 3
    D = steps_D(p, T)
    announce(f"  D per step {np.round(D, 3)}")
    assert all(1.1 <= d <= 1.9 for d in D), D
    check_all([p], T)


def test_2d_scatter_every_step():
    p = pair((48, 56), 2.0, 210.0)
    T = 3
    D = steps_D(p, T)
    announce(f"  D per step {np.round(D, 3)}")
    assert all(d >= 2.1 for d in D), D
    check_all([p], T)


def test_2d_general_gather_then_scatter():
    """Steps of one trajectory on both sides of the 2 px bound: the
    accumulator the scatter adds into must be cleared exactly when the next
    adjoint step scatters."""
    p = pair((48, 56), 2.0, 157.0)
    T = 3
    D = steps_D(p, T)
    announce(f"  D per step {np.round(D, 3)}")
    assert any(1.1 <= d <= 1.9 for d in D) and any(d >= 2.1 for d in D), D
    check_all([p], T)


@pytest.mark.parametrize("shape,sigma,amp", [((14, 18, 22), 1.5, 195.0), ((20, 26, 30), 2.0, 200.0)])
def test_3d_lds_scatter_every_step(shape, sigma, amp):
    p = pair(shape, sigma, amp)
    T = 3
    D = steps_D(p, T)
    announce(f"  D per step {np.round(D, 3)}")
    assert all(1.1 <= d <= 1.97 for d in D), D
    check_all([p], T)


def test_3d_lds3_scatter_every_step():
    p = pair((20, 26, 30), 2.0, 220.0)
    T = 2
    D = steps_D(p, T)
    announce(f"  D per step {np.round(D, 3)}")
    assert all(2.05 <= d <= 2.95 for d in D), D
    check_all([p], T)


def test_3d_global_scatter_every_step():
    p = pair((20, 26, 30), 2.0, 330.0)
    T = 2
    D = steps_D(p, T)
    announce(f"  D per step {np.round(D, 3)}")
    assert all(d >= 3.05 for d in D), D
    check_all([p], T)


def test_3d_lds2_then_lds3_scatter():
    """Steps on both sides of the 2-voxel bound: the two LDS boxes' flushes add
    into the same cleared accumulator."""
    p = pair((14, 18, 22), 1.5, 230.0)
    T = 3
    D = steps_D(p, T)
    announce(f"  D per step {np.round(D, 3)}")
    assert any(1.1 <= d <= 1.95 for d in D) and any(2.05 <= d <= 2.95 for d in D), D
    check_all([p], T)


def test_3d_lds3_then_global_scatter():
    """Steps on both sides of the 3-voxel bound: the LDS box's flush and the
    per-corner atomics add into the same cleared accumulator."""
    p = pair((20, 26, 30), 2.0, 320.0)
    T = 3
    D = steps_D(p, T)
    announce(f"  D per step {np.round(D, 3)}")
    assert any(2.02 <= d <= 2.95 for d in D) and any(d >= 3.05 for d in D), D
    check_all([p], T)


def test_3d_gather_then_scatter():
    p = pair((14, 18, 22), 1.5, 183.5)
    T = 4
    D = steps_D(p, T)
    announce(f"  D per step {np.round(D, 3)}")
    assert any(d <= 0.98 for d in D) and any(d >= 1.05 for d in D), D
    check_all([p], T)


@pytest.mark.parametrize("amp", [None, 195.0])
def test_3d_forced_global_scatter(amp):
    """SHOOT_FORCE_GLOBAL_SCATTER in 3-D, below (realistic momentum) and above
    the one-voxel bound."""
    if amp is None:
        p = G.small_pair((18, 22, 27), 32, rho=0.4, sigma=2.0)
        T = 4
        assert max(steps_D(p, T)) < 1.0
    else:
        p = pair((14, 18, 22), 1.5, amp)
        T = 3
    check_all([p], T, flags=SHOOT_FORCE_GLOBAL_SCATTER)


def test_2d_forced_global_scatter_general_range():
    p = pair((48, 56), 2.0, 120.0)
    check_all([p], 3, flags=SHOOT_FORCE_GLOBAL_SCATTER)


def test_batched_pairs_on_different_paths():
    """One 2-D plan whose pairs take the 3x3 gather, the general gather and the
    scatter, and one 3-D plan whose volumes take the gather, the LDS scatter
    over P +- 2, and the one over P +- 3 then the global scatter: the path is
    chosen per pair inside each launch."""
    T = 3
    p2 = [G.small_pair((40, 52), 7, rho=0.5, sigma=2.0), pair((48, 56), 2.0, 120.0), pair((37, 61), 2.0, 250.0, 9)]
    D2 = [max(steps_D(p, T)) for p in p2]
    announce(f"  2-D max D {np.round(D2, 3)}")
    assert D2[0] < 0.9 and 1.1 <= D2[1] <= 1.9 and min(steps_D(p2[2], T)) >= 2.1
    check_all(p2, T)
    p3 = [G.small_pair((12, 17, 21), 8, rho=0.5, sigma=1.5), pair((14, 18, 22), 1.5, 195.0),
          pair((20, 26, 30), 2.0, 320.0)]
    assert max(steps_D(p3[0], T)) < 0.9
    assert 1.1 <= min(steps_D(p3[1], T)) and max(steps_D(p3[1], T)) <= 1.97
    D3 = steps_D(p3[2], T)
    assert min(D3) >= 2.02 and any(d <= 2.95 for d in D3) and max(D3) >= 3.05, D3
    check_all(p3, T)
