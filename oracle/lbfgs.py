"""L-BFGS on p0 for every pair (TEST INFRASTRUCTURE ONLY, like the rest of
oracle/): the paper's alternative to gradient descent for minimising the
registration cost (Results: the library offers L-BFGS besides gradient
descent). Plain NumPy float64; the algorithm is the textbook limited-memory
BFGS two-loop recursion with Armijo backtracking, with the conventions below
fixed so that the HIP library can follow the same steps:

* history of at most m pairs (s, y); a new pair is always stored, with
  rho = 1 / (s.y) when s.y > 0 and rho = 0 otherwise (such a pair then
  contributes nothing to the recursion);
* the initial inverse Hessian is gamma Id with gamma = s.y / y.y of the
  newest stored pair when its rho > 0, the previous gamma otherwise, and
  1 / ||g|| before any pair exists (a first step of unit length);
* d = -H g; if g.d >= 0, d = -g / ||g|| instead;
* Armijo backtracking from t = 1, halving, at most `trials` evaluations,
  acceptance H(x + t d) <= H(x) + c1 t g.d; when no trial is accepted the
  pair stays at x and its history is cleared (gamma = 1 / ||g||).

Pins (tests/test_oracle_lbfgs.py): the two-loop recursion equals the
explicit product of the BFGS inverse-Hessian updates; on a strictly convex
quadratic the iteration converges to the minimiser.
"""
from typing import Callable, List, Tuple

import numpy as np

from .shooting import cost_and_grad


def two_loop(g: np.ndarray, S: List[np.ndarray], Y: List[np.ndarray], rhos: List[float],
             gamma: float) -> np.ndarray:
    """H g for the L-BFGS inverse Hessian H built from gamma Id and the pairs
    (S[i], Y[i], rhos[i]), oldest first (Nocedal & Wright, Algorithm 7.4)."""
    q = np.array(g, dtype=np.float64, copy=True)
    alphas = []
    for s, y, r in zip(reversed(S), reversed(Y), reversed(rhos)):
        a = r * float(np.vdot(s, q))
        alphas.append(a)
        q = q - a * y
    q = gamma * q
    for (s, y, r), a in zip(zip(S, Y, rhos), reversed(alphas)):
        b = r * float(np.vdot(y, q))
        q = q + (a - b) * s
    return q


def minimize(fg: Callable[[np.ndarray], Tuple[float, np.ndarray]], x0: np.ndarray, iters: int, m: int = 5,
             c1: float = 1e-4, trials: int = 8):
    """L-BFGS with the conventions of the module docstring on one objective.
    Returns (x, history of f at the start of each iteration, trial counts)."""
    x = np.array(x0, dtype=np.float64, copy=True)
    f, g = fg(x)
    S, Y, R = [], [], []
    gamma = 1.0 / max(float(np.linalg.norm(g)), 1e-300)
    hist, used = [], []
    for _ in range(iters):
        hist.append(f)
        d = -two_loop(g, S, Y, R, gamma)
        gd = float(np.vdot(g, d))
        if not gd < 0.0:
            gn = max(float(np.linalg.norm(g)), 1e-300)
            d = -g / gn
            gd = -gn
        t, ok, n = 1.0, False, 0
        for _ in range(trials):
            n += 1
            ft, gt = fg(x + t * d)
            if ft <= f + c1 * t * gd:
                ok = True
                break
            t *= 0.5
        used.append(n)
        if not ok:
            S, Y, R = [], [], []
            gamma = 1.0 / max(float(np.linalg.norm(g)), 1e-300)
            continue
        s = t * d
        y = gt - g
        sy, yy = float(np.vdot(s, y)), float(np.vdot(y, y))
        S.append(s)
        Y.append(y)
        R.append(1.0 / sy if sy > 0.0 else 0.0)
        if len(S) > m:
            S, Y, R = S[1:], Y[1:], R[1:]
        if sy > 0.0 and yy > 0.0:
            gamma = sy / yy
        x, f, g = x + s, ft, gt
    return x, hist, used


def lbfgs(S_img, J, p0, rho: float, sigma: float, lam: float, T: int, iters: int, m: int = 5,
          c1: float = 1e-4, trials: int = 8):
    """L-BFGS on p0 of one pair with the registration cost and its exact
    discrete gradient (cost_and_grad)."""
    def fg(p):
        H, g, _, _ = cost_and_grad(S_img, J, p, rho, sigma, lam, T)
        return H, g
    return minimize(fg, p0, iters, m, c1, trials)
