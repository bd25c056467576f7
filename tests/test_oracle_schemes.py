"""Pins of the Eulerian and mixed schemes (the integration options the paper
compares with the full semi-Lagrangian scheme), and the stability behaviour
the paper reports."""
import numpy as np
import pytest

import oracle as O
import synthetic as G
from golden_fixtures import fig1_steps

T_EUL, T_SL = fig1_steps()  # the paper's Fig. 1 time steps (tests/golden)


@pytest.mark.parametrize("scheme", ["eulerian", "mixed"])
def test_zero_momentum_is_identity(scheme):
    p = G.small_pair((21, 26), seed=51, rho=0.5, sigma=2.0, p0_kind="zero")
    tr = O.shoot(p.source, p.p0, p.rho, p.sigma, 7, scheme=scheme)
    np.testing.assert_array_equal(tr.I[-1], p.source.astype(np.float64))
    np.testing.assert_array_equal(tr.z[-1], np.zeros(p.shape))


@pytest.mark.parametrize("fn", [O.step_eulerian_given_v, O.step_mixed_given_v])
def test_constant_velocity_transports_affine_fields_exactly(fn):
    """rho = 0, constant v, affine I and z: the exact solution is the shift
    I(x - v dt), z(x - v dt) (transport and continuity coincide for constant
    v); both steps reproduce it at points whose stencils stay inside."""
    ny, nx = 20, 24
    q = O.grid_coords((ny, nx))
    I = 0.3 + 0.02 * q[0] - 0.015 * q[1]
    z = -0.1 + 0.01 * q[0] + 0.03 * q[1]
    v = [np.full((ny, nx), 0.7), np.full((ny, nx), -0.4)]
    dt = 0.25
    I1, z1 = fn(I, z, v, 0.0, dt)
    shift = lambda f0, a, b: f0 + a * (-dt * v[0]) + b * (-dt * v[1])  # noqa: E731
    inner = (slice(2, -2), slice(2, -2))
    np.testing.assert_allclose(I1[inner], shift(I, 0.02, -0.015)[inner], rtol=0, atol=1e-13)
    np.testing.assert_allclose(z1[inner], shift(z, 0.01, 0.03)[inner], rtol=0, atol=1e-13)


def test_eulerian_time_stepping_is_first_order():
    """Explicit Euler in time: halving dt halves the change of the result
    (Cauchy ratios of successive refinements tend to 1/2)."""
    p = G.small_pair((32, 32), seed=52, rho=0.4, sigma=3.0, p0_kind="realistic", amplitude=4.0)
    prev, diffs = None, []
    for T in (16, 32, 64, 128):
        a = O.shoot(p.source, p.p0, p.rho, p.sigma, T, scheme="eulerian").I[-1]
        if prev is not None:
            diffs.append(np.linalg.norm(a - prev))
        prev = a
    ratios = [diffs[i + 1] / diffs[i] for i in range(len(diffs) - 1)]
    assert all(abs(r - 0.5) < 0.03 for r in ratios), ratios


def total_variation(f):
    return sum(float(np.abs(np.diff(f, axis=a)).sum()) for a in range(f.ndim))


def test_eulerian_ripples_where_semi_lagrangian_does_not():
    """The stability claim of the Results (Fig. 1), rerun on a synthetic
    LDDMM shot (rho = 0): the semi-Lagrangian image stays within the source's
    range (convex re-interpolation) at dt = 1/20, while the Eulerian scheme at
    the smaller dt = 1/38 overshoots it (ripples); the scheme with only the
    advection semi-Lagrangian (mixed) keeps the image in range but its
    momentum ripples (far larger total variation than the full scheme's)."""
    S, J, p0 = G.ripple_case()
    sl = O.shoot(S, p0, 0.0, 3.0, T_SL, scheme="sl")
    eu = O.shoot(S, p0, 0.0, 3.0, T_EUL, scheme="eulerian")
    mx = O.shoot(S, p0, 0.0, 3.0, T_SL, scheme="mixed")
    lo, hi = float(S.min()), float(S.max())
    over = lambda I: max(float(I.max()) - hi, lo - float(I.min()), 0.0)  # noqa: E731
    assert over(sl.I[-1]) == 0.0
    assert over(eu.I[-1]) > 0.1
    assert over(mx.I[-1]) == 0.0
    assert total_variation(mx.z[-1]) > 1.2 * total_variation(sl.z[-1])


def test_eulerian_integration_fails_where_semi_lagrangian_holds():
    """Twice the momentum: the Eulerian shot at dt = 1/38 diverges (the
    integration fails), the semi-Lagrangian one at dt = 1/20 stays finite and
    within range."""
    S, J, p0 = G.ripple_case(amplitude=200.0)
    with np.errstate(all="ignore"):
        eu = O.shoot(S, p0, 0.0, 3.0, T_EUL, scheme="eulerian").I[-1]
    sl = O.shoot(S, p0, 0.0, 3.0, T_SL, scheme="sl").I[-1]
    assert not np.all(np.isfinite(eu))
    assert np.all(np.isfinite(sl)) and sl.max() <= S.max() and sl.min() >= S.min()
