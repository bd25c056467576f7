"""Pins of the oracle's deformation map psi_T (psi_0 = Id, psi_{t+1} =
psi_t o (Id - dt v_t) by the scheme's clamped multilinear re-interpolation)."""
import numpy as np
import pytest

import oracle as O
import synthetic as G


@pytest.mark.parametrize("shape", [(20, 27), (7, 9, 8)])
def test_zero_momentum_gives_the_identity_map(shape):
    p = G.small_pair(shape, seed=11, rho=0.5, sigma=1.5, p0_kind="zero")
    psi = O.deformation(p.source, p.p0, p.rho, p.sigma, T=4)
    np.testing.assert_array_equal(psi, O.grid_coords(shape))


@pytest.mark.parametrize("shape,amp", [((24, 30), 120.0), ((9, 11, 10), 300.0)])
def test_one_step_is_the_clamped_foot(shape, amp):
    """T = 1: interpolating the identity at a foot returns the foot clamped
    into the grid, psi_1 = clip(q - v_0, 0, n - 1); the momentum is large
    enough that feet span several cells and leave the grid."""
    p = G.small_pair(shape, seed=12, rho=0.5, sigma=1.5, p0_kind="realistic", amplitude=amp)
    traj = O.shoot(p.source, p.p0, p.rho, p.sigma, 1)
    q = O.grid_coords(shape)
    y = np.stack([q[a] - traj.v[0][a] for a in range(len(shape))])
    assert np.max(np.abs(y - q)) > 2.0
    assert any(y[a].min() < 0 or y[a].max() > n - 1 for a, n in enumerate(shape))
    want = np.stack([np.clip(y[a], 0.0, n - 1.0) for a, n in enumerate(shape)])
    psi = O.deformation(p.source, p.p0, p.rho, p.sigma, 1, traj=traj)
    np.testing.assert_allclose(psi, want, rtol=0, atol=1e-12)


def test_one_step_map_transports_the_source():
    """rho = 0, T = 1: the image is the source at the feet, and so is the
    source re-interpolated at psi_1 (the same clamped feet)."""
    shape = (26, 22)
    p = G.small_pair(shape, seed=13, rho=0.0, sigma=2.0, p0_kind="realistic", amplitude=30.0)
    traj = O.shoot(p.source, p.p0, 0.0, p.sigma, 1)
    psi = O.deformation(p.source, p.p0, 0.0, p.sigma, 1, traj=traj)
    np.testing.assert_allclose(O.interp(p.source, O.feet(psi, shape)), traj.I[1], rtol=0, atol=1e-12)


def test_no_velocity_keeps_the_identity_over_many_steps():
    """A constant source with rho = 0 never moves (grad I = 0 gives v_t = 0
    for every t, whatever p0), so psi_T is the identity although p0 != 0."""
    shape = (18, 23)
    p = G.small_pair(shape, seed=14, rho=0.0, sigma=2.0, p0_kind="random")
    S = np.full(shape, 0.7)
    psi = O.deformation(S, p.p0, 0.0, p.sigma, T=6)
    assert np.max(np.abs(p.p0)) > 0
    np.testing.assert_array_equal(psi, O.grid_coords(shape))


def test_first_step_leaves_a_still_axis_unchanged():
    """Source and momentum constant along x: D_x I = 0, so v_x = 0 at the
    first step and the x component of psi_1 is x (to rounding) while y moves."""
    ny, nx = 30, 17
    yy = np.arange(ny, dtype=np.float64)[:, None] * np.ones((1, nx))
    S = 0.5 + 0.4 * np.sin(yy / 4.0)
    p0 = 3.0 * np.cos(yy / 5.0)
    psi = O.deformation(S, p0, 0.3, 2.0, T=1)
    q = O.grid_coords((ny, nx))
    np.testing.assert_allclose(psi[1], q[1], rtol=0, atol=1e-12)   # (1 - f) x + f x, rounded
    assert np.max(np.abs(psi[0] - q[0])) > 0.1
    assert psi[0].min() >= 0.0 and psi[0].max() <= ny - 1.0
