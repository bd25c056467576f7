"""Pins of the oracle's gradient-descent driver and energy diagnostic against
closed forms (no GPU).

Gradient descent (Results: every cost is minimised by gradient descent). With a
constant source S = c and T = 1 the velocity is zero (D c = 0), every foot sits
on its arrival point, and one step gives I_1 = c + rho p0. The cost of Eq. 4 is
then the separable quadratic

    H(p) = 1/2 ||rho p - (J - c)||^2 + lambda rho ||p||^2
         = H* + a/2 ||p - p*||^2,  a = rho^2 + 2 lambda rho,  p* = rho (J - c) / a,

so a descent step p <- p - eta dH/dp multiplies the error e = p - p* by
(1 - eta a): the iterates, the costs and the step-halving decisions (the step
is halved when the cost at the current iterate exceeds the previous one) all
follow from the scalar sequence of |1 - eta_k a| alone.
"""
import numpy as np

import oracle as O


def _quadratic_case(shape=(9, 11), c=0.3, rho=0.5, lam=0.01, seed=5):
    rng = np.random.default_rng(seed)
    S = np.full(shape, c)
    J = c + rng.normal(0.0, 0.2, size=shape)
    p0 = rng.normal(0.0, 0.5, size=shape)
    a = rho * rho + 2.0 * lam * rho
    p_star = rho * (J - c) / a
    H_star = 0.5 * np.sum((rho * p_star - (J - c)) ** 2) + lam * rho * np.sum(p_star ** 2)
    return S, J, p0, rho, lam, a, p_star, H_star


def test_cost_is_the_closed_form_quadratic():
    S, J, p0, rho, lam, a, p_star, H_star = _quadratic_case()
    H, g, _, _ = O.cost_and_grad(S, J, p0, rho, 2.0, lam, 1)
    assert abs(H - (H_star + 0.5 * a * np.sum((p0 - p_star) ** 2))) <= 1e-12 * H
    np.testing.assert_allclose(g, a * (p0 - p_star), rtol=0, atol=1e-13)


def _expected_descent(p0, p_star, H_star, a, eta, iters):
    """Iterates and costs of the halving rule, from e_{k+1} = (1 - eta_k a) e_k."""
    e = p0 - p_star
    costs, etas = [], []
    prev = None
    for _ in range(iters):
        Hk = H_star + 0.5 * a * np.sum(e * e)
        if prev is not None and Hk > prev:
            eta *= 0.5
        costs.append(Hk)
        etas.append(eta)
        prev = Hk
        e = (1.0 - eta * a) * e
    return p_star + e, costs, etas


def test_descent_step_and_halving_follow_the_closed_form():
    S, J, p0, rho, lam, a, p_star, H_star = _quadratic_case()
    # eta0 a = 2.6: the first step overshoots (|1 - eta a| = 1.6), the cost
    # rises, the step is halved once (|1 - eta a| = 0.3) and then decreases
    eta0 = 10.0
    assert abs(1.0 - eta0 * a) > 1.0 and abs(1.0 - 0.5 * eta0 * a) < 1.0
    iters = 6
    p, hist = O.gradient_descent(S, J, p0, rho, 2.0, lam, 1, iters=iters, eta=eta0)
    p_ref, costs, etas = _expected_descent(p0, p_star, H_star, a, eta0, iters)
    assert etas[:2] == [eta0, 0.5 * eta0] and len(set(etas[1:])) == 1
    np.testing.assert_allclose(hist, costs, rtol=1e-12)
    np.testing.assert_allclose(p, p_ref, rtol=0, atol=1e-11)


def test_one_descent_step_is_p_minus_eta_grad():
    S, J, p0, rho, lam, a, p_star, _ = _quadratic_case(seed=9)
    eta = 0.7
    p, hist = O.gradient_descent(S, J, p0, rho, 2.0, lam, 1, iters=1, eta=eta)
    np.testing.assert_allclose(p, p0 - eta * a * (p0 - p_star), rtol=0, atol=1e-13)
    assert len(hist) == 1


def test_halving_repeats_while_the_cost_keeps_rising():
    S, J, p0, rho, lam, a, p_star, H_star = _quadratic_case(seed=11)
    # eta a = 10.4, 5.2 and 2.6 overshoot (the step is halved at each of the
    # next three iterations), 1.3 converges
    eta0 = 40.0
    iters = 7
    p, hist = O.gradient_descent(S, J, p0, rho, 2.0, lam, 1, iters=iters, eta=eta0)
    p_ref, costs, etas = _expected_descent(p0, p_star, H_star, a, eta0, iters)
    assert etas == [eta0, eta0 / 2, eta0 / 4, eta0 / 8] + [eta0 / 8] * (iters - 4)
    np.testing.assert_allclose(hist, costs, rtol=1e-12)
    np.testing.assert_allclose(p, p_ref, rtol=0, atol=1e-9)


# ---------------------------------------------------------------- energy

def test_energy_of_a_constant_image_is_rho_norm():
    """D c = 0, so m = 0 and ||v||_V^2 vanishes: only rho ||z||^2 is left."""
    rng = np.random.default_rng(3)
    z = rng.normal(size=(12, 15))
    w = O.gaussian_taps(1.7)
    assert abs(O.energy(np.full((12, 15), 0.4), z, 0.6, w) - 0.6 * np.sum(z * z)) <= 1e-12 * np.sum(z * z)


def test_energy_of_an_impulse_on_a_ramp():
    """z = a unit impulse at an interior point q of a ramp I = s0 y + s1 x:
    m_a = s_a delta_q (central differences are exact on a ramp away from the
    edges), so <m, G m> = (s0^2 + s1^2) G[q, q] with G[q, q] = w_0^2, the
    product of the centre taps of the two axis passes."""
    shape = (21, 23)
    sigma = 1.3
    s0, s1 = 0.7, -0.4
    yy, xx = np.meshgrid(np.arange(shape[0], dtype=float), np.arange(shape[1], dtype=float), indexing="ij")
    I = s0 * yy + s1 * xx
    z = np.zeros(shape)
    z[10, 11] = 1.0
    w = O.gaussian_taps(sigma)
    r = int(np.floor(3 * sigma))
    w0 = 1.0 / sum(np.exp(-k * k / (2 * sigma * sigma)) for k in range(-r, r + 1))
    rho = 0.25
    ref = (s0 * s0 + s1 * s1) * w0 * w0 + rho
    assert abs(O.energy(I, z, rho, w) - ref) <= 1e-13
