"""Pins of the oracle's hand-written discrete adjoint: central finite
differences of the cost and torch autograd of an independent float64 program."""
import numpy as np
import pytest

import oracle as O
import synthetic as G

from torch_program import cost_and_grad as torch_cost_and_grad


def _min_distance_to_grid_lines(pair, T):
    tr = O.shoot(pair.source, pair.p0, pair.rho, pair.sigma, T)
    q = O.grid_coords(pair.shape)
    dt = 1.0 / T
    m = np.inf
    for v in tr.v:
        for a in range(pair.ndim):
            y = q[a] - dt * v[a]
            inside = (y > 0) & (y < pair.shape[a] - 1)
            if inside.any():
                m = min(m, np.abs(y - np.round(y))[inside].min())
    return m


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_full_gradient_central_fd_16x16():
    """Every component of dH/dp0 against central differences on a 16x16 pair
    (realistic momentum, no foot crosses a grid line under the perturbation)."""
    pair = G.small_pair((16, 16), 11, rho=0.5, sigma=2.0)
    T = 5
    S, J, p0 = (x.astype(np.float64) for x in (pair.source, pair.target, pair.p0))
    assert _min_distance_to_grid_lines(pair, T) > 1e-7  # perturbations move feet ~1e-8 px
    H, g, _, _ = O.cost_and_grad(S, J, p0, pair.rho, pair.sigma, pair.lam, T)
    h = 1e-6
    fd = np.zeros_like(p0)
    for idx in np.ndindex(p0.shape):
        e = np.zeros_like(p0)
        e[idx] = h
        fd[idx] = (O.cost(S, J, p0 + e, pair.rho, pair.sigma, pair.lam, T)
                   - O.cost(S, J, p0 - e, pair.rho, pair.sigma, pair.lam, T)) / (2 * h)
    assert _rel(g, fd) <= 1e-7


def test_full_gradient_central_fd_3d():
    """Every component of dH/dp0 against central differences on a 6x7x5 volume."""
    pair = G.small_pair((6, 7, 5), 12, rho=0.4, sigma=1.2)
    T = 4
    S, J, p0 = (x.astype(np.float64) for x in (pair.source, pair.target, pair.p0))
    assert _min_distance_to_grid_lines(pair, T) > 1e-7
    _, g, _, _ = O.cost_and_grad(S, J, p0, pair.rho, pair.sigma, pair.lam, T)
    h = 1e-6
    fd = np.zeros_like(p0)
    for idx in np.ndindex(p0.shape):
        e = np.zeros_like(p0)
        e[idx] = h
        fd[idx] = (O.cost(S, J, p0 + e, pair.rho, pair.sigma, pair.lam, T)
                   - O.cost(S, J, p0 - e, pair.rho, pair.sigma, pair.lam, T)) / (2 * h)
    assert _rel(g, fd) <= 1e-7


@pytest.mark.parametrize("kind", ["zero", "random", "realistic"])
@pytest.mark.parametrize("shape,T,sigma,rho", [((12, 15), 4, 1.5, 0.6), ((5, 7, 6), 3, 1.0, 0.3),
                                               ((10, 10), 2, 2.0, 0.0)])
def test_gradient_matches_independent_autograd(kind, shape, T, sigma, rho):
    """Hand-written adjoint == torch autograd of an independent float64
    program, including p0 = 0 where every foot lies on the grid."""
    pair = G.small_pair(shape, 21, rho=rho, sigma=sigma, p0_kind=kind)
    S, J, p0 = (x.astype(np.float64) for x in (pair.source, pair.target, pair.p0))
    H, g, _, _ = O.cost_and_grad(S, J, p0, pair.rho, pair.sigma, pair.lam, T)
    Ht, gt = torch_cost_and_grad(S, J, p0, pair.rho, pair.sigma, pair.lam, T)
    assert abs(H - Ht) <= 1e-12 * abs(Ht)
    assert _rel(g, gt) <= 1e-11


def test_gradient_at_zero_momentum_matches_autograd_on_disk():
    """The GD starting point (p0 = 0) of the 64x64 disk workload."""
    pair = G.disk_pair(1, "zero")
    S, J, p0 = (x.astype(np.float64) for x in (pair.source, pair.target, pair.p0))
    H, g, _, _ = O.cost_and_grad(S, J, p0, pair.rho, pair.sigma, pair.lam, 10)
    Ht, gt = torch_cost_and_grad(S, J, p0, pair.rho, pair.sigma, pair.lam, 10)
    assert abs(H - Ht) <= 1e-12 * Ht
    assert _rel(g, gt) <= 1e-11


def test_gradient_descent_decreases_cost():
    pair = G.small_pair((20, 20), 2, rho=0.5, sigma=2.0, p0_kind="zero")
    p, hist = O.gradient_descent(pair.source, pair.target, pair.p0, pair.rho, pair.sigma,
                                 pair.lam, 4, iters=5)
    assert hist[-1] < hist[0]
