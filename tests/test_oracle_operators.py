"""Pins of the oracle's operators against library routines, closed forms and
invariants (CPU only)."""
import itertools

import numpy as np
import pytest
import torch
from scipy import ndimage

import oracle as O

RNG = np.random.default_rng(1234)


# --- Gaussian kernel K ------------------------------------------------------

@pytest.mark.parametrize("sigma", [1.0, 2.0, 2.1, 3.0, 4.0, 5.0, 6.0])
def test_taps_match_scipy_gaussian_filter(sigma):
    """Where floor(3 sigma) equals SciPy's round(3 sigma) radius, the taps
    equal SciPy's own normalised Gaussian: gaussian_filter1d of a unit impulse."""
    r = int(np.floor(3 * sigma))
    assert r == int(3.0 * sigma + 0.5)
    w = O.gaussian_taps(sigma)
    assert w.shape == (2 * r + 1,)
    impulse = np.zeros(4 * r + 3)
    impulse[2 * r + 1] = 1.0
    ref = ndimage.gaussian_filter1d(impulse, sigma, truncate=3.0, mode="constant")
    np.testing.assert_allclose(w, ref[r + 1: 3 * r + 2], rtol=0, atol=1e-15)


@pytest.mark.parametrize("sigma", [2.5, 2.3333, 4.9])
def test_taps_truncation_and_normalisation(sigma):
    w = O.gaussian_taps(sigma)
    r = (len(w) - 1) // 2
    assert r == int(np.floor(3 * sigma))
    assert abs(w.sum() - 1.0) < 1e-15
    np.testing.assert_array_equal(w, w[::-1])
    k = np.arange(-r, r + 1)
    ratio = w / w[r]
    np.testing.assert_allclose(ratio, np.exp(-k ** 2 / (2 * sigma ** 2)), rtol=1e-14)


@pytest.mark.parametrize("shape", [(17, 23), (9, 12, 14)])
def test_conv_axis_matches_correlate1d(shape):
    f = RNG.standard_normal(shape)
    w = O.gaussian_taps(1.7)
    for a in range(len(shape)):
        ref = ndimage.correlate1d(f, w, axis=a, mode="constant", cval=0.0)
        np.testing.assert_allclose(O.conv_axis(f, w, a), ref, rtol=0, atol=1e-14)


def test_smooth_preserves_constants_away_from_edges():
    w = O.gaussian_taps(2.0)
    r = (len(w) - 1) // 2
    f = np.full((30, 31), 3.25)
    g = O.smooth(f, w)
    np.testing.assert_allclose(g[r:-r, r:-r], 3.25, rtol=1e-14)
    assert g[0, 0] < 3.25  # zero padding bites at the border


def test_smooth_self_adjoint():
    w = O.gaussian_taps(2.3)
    a = RNG.standard_normal((20, 26))
    b = RNG.standard_normal((20, 26))
    lhs = np.sum(O.smooth(a, w) * b)
    rhs = np.sum(a * O.smooth(b, w))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


# --- central differences ----------------------------------------------------

def test_diff_exact_on_affine_interior_and_one_sided_at_edges():
    n0, n1 = 11, 13
    yy, xx = np.meshgrid(np.arange(n0), np.arange(n1), indexing="ij")
    f = 3.0 * xx - 2.0 * yy + 1.0
    dx = O.diff(f, 1)
    dy = O.diff(f, 0)
    np.testing.assert_allclose(dx[:, 1:-1], 3.0, rtol=1e-15)
    np.testing.assert_allclose(dy[1:-1, :], -2.0, rtol=1e-15)
    np.testing.assert_allclose(dx[:, 0], 1.5)       # (f[1] - f[0]) / 2
    np.testing.assert_allclose(dx[:, -1], 1.5)
    np.testing.assert_allclose(dy[0, :], -1.0)


@pytest.mark.parametrize("n", [2, 3, 7])
def test_diff_T_dot_product_and_closed_form(n):
    g = RNG.standard_normal((n, 5))
    f = RNG.standard_normal((n, 5))
    lhs = np.sum(O.diff(f, 0) * g)
    rhs = np.sum(f * O.diff_T(g, 0))
    assert abs(lhs - rhs) <= 1e-14 * max(1.0, abs(lhs))
    # closed form of the transpose rows
    dt = O.diff_T(g, 0)
    ref = np.empty_like(g)
    for j in range(n):
        if j == 0:
            ref[j] = -0.5 * (g[0] + g[1])
        elif j == n - 1:
            ref[j] = 0.5 * (g[n - 2] + g[n - 1])
        else:
            ref[j] = 0.5 * (g[j - 1] - g[j + 1])
    np.testing.assert_allclose(dt, ref, rtol=0, atol=1e-15)


# --- interpolation ------------------------------------------------------------

def _feet_from(y, shape):
    return O.feet(y, shape)


@pytest.mark.parametrize("shape", [(13, 17), (6, 9, 11)])
def test_interp_matches_map_coordinates(shape):
    F = RNG.standard_normal(shape)
    y = np.stack([RNG.uniform(-2.0, n + 1.0, size=shape) for n in shape])
    ref = ndimage.map_coordinates(F, y.reshape(len(shape), -1), order=1, mode="nearest")
    got = O.interp(F, O.feet(y, shape)).reshape(-1)
    np.testing.assert_allclose(got, ref, rtol=0, atol=2e-15)


@pytest.mark.parametrize("shape", [(13, 17), (6, 9, 11)])
def test_interp_and_grad_match_grid_sample(shape):
    """torch grid_sample(border, align_corners=True) in float64, values and
    autograd derivative w.r.t. the coordinates at generic (non-integer) points."""
    d = len(shape)
    F = RNG.standard_normal(shape)
    y = np.stack([RNG.uniform(-1.5, n + 0.5, size=shape) for n in shape])
    ft = O.feet(y, shape)
    val = O.interp(F, ft)
    grads = O.interp_grad(F, ft)
    # grid_sample wants (x, y[, z]) = reversed axes, normalised to [-1, 1]
    yt = torch.tensor(y, requires_grad=True)
    norm = [2.0 * yt[a] / (shape[a] - 1) - 1.0 for a in range(d)]
    grid = torch.stack(norm[::-1], dim=-1).unsqueeze(0)
    Ft = torch.tensor(F).unsqueeze(0).unsqueeze(0)
    out = torch.nn.functional.grid_sample(Ft, grid, mode="bilinear", padding_mode="border",
                                          align_corners=True).reshape(shape)
    np.testing.assert_allclose(val, out.detach().numpy(), rtol=0, atol=1e-13)
    out.sum().backward()
    for a in range(d):
        np.testing.assert_allclose(grads[a], yt.grad[a].numpy(), rtol=0, atol=1e-12)


def test_interp_integer_shift_is_exact_with_edge_replication():
    F = RNG.standard_normal((9, 12))
    q = O.grid_coords(F.shape)
    y = q.copy()
    y[1] -= 2.0   # sample two pixels to the left: shift right by 2
    y[0] += 1.0   # one row down: shift up by 1
    got = O.interp(F, O.feet(y, F.shape))
    ref = F[np.clip(np.arange(9) + 1, 0, 8)][:, np.clip(np.arange(12) - 2, 0, 11)]
    np.testing.assert_array_equal(got, ref)


def test_interp_reproduces_affine_fields_inside():
    shape = (10, 14, 9)
    q = O.grid_coords(shape)
    F = 0.5 + 2.0 * q[0] - 1.25 * q[1] + 0.75 * q[2]
    y = np.stack([RNG.uniform(0.0, n - 1.0, size=shape) for n in shape])
    got = O.interp(F, O.feet(y, shape))
    np.testing.assert_allclose(got, 0.5 + 2.0 * y[0] - 1.25 * y[1] + 0.75 * y[2], rtol=0, atol=1e-13)
    g = O.interp_grad(F, O.feet(y, shape))
    for a, c in enumerate((2.0, -1.25, 0.75)):
        np.testing.assert_allclose(g[a], c, rtol=1e-13)


def test_interp_grad_is_central_fd_of_interp():
    shape = (8, 11)
    F = RNG.standard_normal(shape)
    y = np.stack([RNG.uniform(0.2, n - 1.2, size=shape) for n in shape])
    # keep away from grid lines so that the FD does not straddle a kink
    y = np.where(np.abs(y - np.round(y)) < 1e-3, y + 0.01, y)
    h = 1e-7
    g = O.interp_grad(F, O.feet(y, shape))
    for a in range(2):
        e = np.zeros_like(y)
        e[a] = h
        fd = (O.interp(F, O.feet(y + e, shape)) - O.interp(F, O.feet(y - e, shape))) / (2 * h)
        np.testing.assert_allclose(g[a], fd, rtol=0, atol=1e-7)


def test_interp_grad_kink_conventions():
    """On a grid line the derivative is the forward difference (cell floor(c));
    at or beyond a border it is zero."""
    F = RNG.standard_normal((5, 6))
    y = O.grid_coords(F.shape).astype(float)
    g = O.interp_grad(F, O.feet(y, F.shape))
    for j in range(1, 5):
        np.testing.assert_allclose(g[1][:, j], F[:, j + 1] - F[:, j])
    np.testing.assert_array_equal(g[1][:, 0], 0.0)
    np.testing.assert_array_equal(g[1][:, 5], 0.0)
    np.testing.assert_array_equal(g[0][0, :], 0.0)
    np.testing.assert_array_equal(g[0][4, :], 0.0)


@pytest.mark.parametrize("shape", [(7, 10), (5, 6, 7), (2, 2)])
def test_interp_T_dot_product(shape):
    F = RNG.standard_normal(shape)
    a = RNG.standard_normal(shape)
    y = np.stack([RNG.uniform(-1.0, n, size=shape) for n in shape])
    ft = O.feet(y, shape)
    lhs = np.sum(O.interp(F, ft) * a)
    rhs = np.sum(F * O.interp_T(a, ft, shape))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


def test_interp_T_conserves_mass():
    """Interpolation weights sum to one, so the transpose keeps the total."""
    shape = (9, 8, 7)
    a = RNG.standard_normal(shape)
    y = np.stack([RNG.uniform(-3.0, n + 2.0, size=shape) for n in shape])
    out = O.interp_T(a, O.feet(y, shape), shape)
    assert abs(out.sum() - a.sum()) < 1e-12


def test_feet_cells_stay_inside_grid():
    shape = (4, 5)
    y = np.stack([np.full(shape, -7.0), np.full(shape, 9.0)])
    ft = O.feet(y, shape)
    np.testing.assert_array_equal(ft.cell[0], 0)
    np.testing.assert_array_equal(ft.frac[0], 0.0)
    np.testing.assert_array_equal(ft.cell[1], 3)
    np.testing.assert_array_equal(ft.frac[1], 1.0)
    for c in itertools.chain(ft.live):
        np.testing.assert_array_equal(c, 0.0)
