"""Pins of the oracle's shooting scheme and cost: invariants, special cases
with closed forms, and the transport sign fixed by the paper's equations."""
import numpy as np
import pytest

import oracle as O
import synthetic as G

RNG = np.random.default_rng(99)


@pytest.mark.parametrize("shape,T", [((16, 19), 4), ((7, 8, 9), 3)])
def test_zero_momentum_is_identity(shape, T):
    """p0 = 0 gives v = 0, I_T = S, z_T = 0 and H = 1/2 ||S - J||^2 exactly."""
    S = RNG.standard_normal(shape)
    J = RNG.standard_normal(shape)
    p0 = np.zeros(shape)
    tr = O.shoot(S, p0, 0.7, 1.5, T)
    np.testing.assert_array_equal(tr.I[-1], S)
    np.testing.assert_array_equal(tr.z[-1], 0.0)
    for v in tr.v:
        for va in v:
            assert np.all(va == 0.0)
    H, data, reg = O.cost_terms(S, J, p0, 0.7, 1.5, 0.01, T)
    assert H == 0.5 * np.sum((S - J) ** 2)
    assert reg == 0.0


@pytest.mark.parametrize("shape", [(12, 15), (6, 7, 8)])
def test_constant_image_lddmm_limit_is_static(shape):
    """Constant S and rho = 0: grad S = 0, so v = 0 at every step; the image
    stays S and the momentum is only carried along (z_T = p0)."""
    S = np.full(shape, 0.37)
    p0 = RNG.standard_normal(shape)
    tr = O.shoot(S, p0, 0.0, 2.0, 5)
    for v in tr.v:
        for va in v:
            assert np.all(va == 0.0)
    np.testing.assert_array_equal(tr.I[-1], S)
    np.testing.assert_array_equal(tr.z[-1], p0)


def test_constant_image_first_velocity_vanishes_for_any_rho():
    S = np.full((10, 11), -1.5)
    p0 = RNG.standard_normal((10, 11))
    tr = O.shoot(S, p0, 0.8, 2.0, 3)
    for va in tr.v[0]:
        assert np.all(va == 0.0)
    assert not np.all(tr.I[1] == S)  # rho dt p0 was added


@pytest.mark.parametrize("shape", [(9, 13), (5, 6, 4)])
def test_constant_image_one_step_closed_form(shape):
    """Constant S = c, T = 1: I_1 = c + rho p0, H = 1/2||I_1 - J||^2 +
    lambda rho ||p0||^2 and dH/dp0 = rho (I_1 - J) + 2 lambda rho p0."""
    c, rho, lam = 0.6, 0.45, 0.03
    S = np.full(shape, c)
    J = RNG.standard_normal(shape)
    p0 = RNG.standard_normal(shape)
    tr = O.shoot(S, p0, rho, 1.3, 1)
    I1 = c + rho * p0
    np.testing.assert_allclose(tr.I[-1], I1, rtol=1e-15, atol=1e-15)
    H, g, _, _ = O.cost_and_grad(S, J, p0, rho, 1.3, lam, 1)
    Href = 0.5 * np.sum((I1 - J) ** 2) + lam * rho * np.sum(p0 ** 2)
    assert abs(H - Href) <= 1e-15 * Href
    np.testing.assert_allclose(g, rho * (I1 - J) + 2 * lam * rho * p0, rtol=1e-14, atol=1e-15)


def test_maximum_principle_without_residual():
    """rho = 0 (pure LDDMM transport): interpolation weights are convex, so
    min S <= I_t <= max S at every step."""
    pair = G.small_pair((20, 24), 3, rho=0.0, sigma=2.0, amplitude=25.0)
    tr = O.shoot(pair.source, pair.p0, 0.0, pair.sigma, 6)
    lo, hi = pair.source.min(), pair.source.max()
    assert O.max_displacement(tr, 6) > 0.05
    for I in tr.I:
        assert I.min() >= lo and I.max() <= hi


def test_integer_velocity_gives_exact_shift():
    """A constant velocity with dt * v = (1, -2) pixels moves the image by
    exactly that amount (the foot is q - dt v); div v = 0 keeps z unchanged
    apart from the same shift."""
    F = RNG.standard_normal((9, 12))
    z = RNG.standard_normal((9, 12))
    dt = 0.25
    v = [np.full(F.shape, 1.0 / dt), np.full(F.shape, -2.0 / dt)]
    I1, z1, aux = O.step_given_v(F, z, v, rho=0.0, dt=dt)
    rows = np.clip(np.arange(9) - 1, 0, 8)
    cols = np.clip(np.arange(12) + 2, 0, 11)
    np.testing.assert_array_equal(I1, F[rows][:, cols])
    np.testing.assert_array_equal(z1, z[rows][:, cols])


def test_transport_sign_on_a_ramp():
    """Eq. 1 with v = -K * (z grad I): for a ramp I = x and z > 0 the transport
    term -<grad I, v> = <grad I, K * (z grad I)> is positive, so with rho = 0
    the image rises in the interior after one step."""
    shape = (24, 40)
    I0 = np.tile(np.arange(shape[1], dtype=float) * 0.1, (shape[0], 1))
    z0 = np.full(shape, 0.5)
    I1, _, aux = O.step(I0, z0, 0.0, 0.1, O.gaussian_taps(2.0))
    assert np.all(aux["v"][1][6:-6, 8:-8] < 0)
    assert np.all(I1[6:-6, 8:-8] > I0[6:-6, 8:-8])


def test_regulariser_is_v0_norm_plus_rho_l2():
    """The regulariser equals <m0, G m0> + rho ||p0||^2 = -<m0, v0> + rho ||p0||^2."""
    pair = G.small_pair((14, 17), 8, rho=0.3, sigma=1.5)
    H, data, reg = O.cost_terms(pair.source, pair.target, pair.p0, pair.rho, pair.sigma,
                                pair.lam, 3)
    tr = O.shoot(pair.source, pair.p0, pair.rho, pair.sigma, 3)
    m0 = O.momentum_field(pair.source, pair.p0)
    ref = -sum(np.sum(m * v) for m, v in zip(m0, tr.v[0])) + pair.rho * np.sum(
        pair.p0.astype(float) ** 2)
    assert abs(reg - pair.lam * ref) <= 1e-12 * abs(reg)
    assert abs(data - 0.5 * np.sum((tr.I[-1] - pair.target) ** 2)) <= 1e-12 * data


def test_energy_drift_is_small_for_small_steps():
    """The discrete energy ||v_t||_V^2 + rho ||z_t||^2 (pinned itself by
    closed forms in test_oracle_descent.py) changes little along the
    shooting: the continuous geodesic conserves it, the discrete scheme only
    approximately, so this is a loose sanity bound, not a parity pin."""
    pair = G.small_pair((32, 32), 4, rho=0.5, sigma=2.0)
    T = 10
    tr = O.shoot(pair.source, pair.p0, pair.rho, pair.sigma, T)
    w = O.gaussian_taps(pair.sigma)
    e = [O.energy(I, z, pair.rho, w) for I, z in zip(tr.I, tr.z)]
    assert max(e) / min(e) < 1.5
