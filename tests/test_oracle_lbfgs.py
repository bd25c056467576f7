"""Pins of the oracle's L-BFGS (oracle/lbfgs.py)."""
import numpy as np

import oracle as O
import synthetic as G


def explicit_inverse_hessian(S, Y, R, gamma, n):
    H = gamma * np.eye(n)
    for s, y, r in zip(S, Y, R):
        V = np.eye(n) - r * np.outer(y, s)
        H = V.T @ H @ V + r * np.outer(s, s)
    return H


def test_two_loop_equals_the_explicit_bfgs_product():
    rng = np.random.default_rng(3)
    n = 7
    B = rng.normal(size=(n, n))
    A = B @ B.T + n * np.eye(n)
    S = [rng.normal(size=n) for _ in range(4)]
    Y = [A @ s for s in S]
    R = [1.0 / float(s @ y) for s, y in zip(S, Y)]
    R[1] = 0.0                    # a stored pair without curvature is a no-op
    g = rng.normal(size=n)
    gamma = 0.37
    H = explicit_inverse_hessian(S, Y, R, gamma, n)
    np.testing.assert_allclose(O.two_loop(g, S, Y, R, gamma), H @ g, rtol=1e-12, atol=1e-13)


def test_converges_on_a_strictly_convex_quadratic():
    rng = np.random.default_rng(4)
    n = 20
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    A = Q @ np.diag(np.linspace(1.0, 50.0, n)) @ Q.T
    b = rng.normal(size=n)

    def fg(x):
        return 0.5 * x @ A @ x - b @ x, A @ x - b

    x, hist, used = O.lbfgs_minimize(fg, np.zeros(n), iters=80, m=6)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-7, atol=1e-9)
    assert all(h1 <= h0 for h0, h1 in zip(hist, hist[1:]))


def test_registration_cost_decreases_monotonically():
    p = G.small_pair((20, 24), seed=31, rho=0.5, sigma=2.0, p0_kind="zero", lam=0.01)
    x, hist, used = O.lbfgs(p.source, p.target, p.p0, p.rho, p.sigma, p.lam, 5, iters=6)
    assert all(h1 <= h0 for h0, h1 in zip(hist, hist[1:]))
    assert hist[-1] < 0.5 * hist[0]
