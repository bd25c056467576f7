"""Helpers of the GPU tests: run plans through the C ABI and compare with the
oracle."""
import sys

import numpy as np
import torch

import oracle
from paper_2106_08817_amd import PairSpec, Plan


def announce(msg: str) -> None:
    sys.__stderr__.write(f"[gpu-case] {msg}\n")
    sys.__stderr__.flush()


def dev(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def specs(pairs):
    return [PairSpec(dev(p.source), dev(p.p0), p.rho, p.sigma, p.lam, dev(p.target)) for p in pairs]


def run(pairs, T, op="grad", flags=0, budget=0):
    plan = Plan(specs(pairs), T, flags, budget)
    getattr(plan, op)()
    torch.cuda.synchronize()
    return plan


def host(t) -> np.ndarray:
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b) -> float:
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def oracle_forward(p, T):
    tr = oracle.shoot(p.source, p.p0, p.rho, p.sigma, T)
    H = oracle.cost_terms(p.source, p.target, p.p0, p.rho, p.sigma, p.lam, T, tr)
    return tr.I[-1], tr.z[-1], H


def oracle_grad(p, T):
    H, g, _, (data, reg) = oracle.cost_and_grad(p.source, p.target, p.p0, p.rho, p.sigma, p.lam, T)
    return H, g, data, reg


IMG_TOL = 1e-5    # final image and momentum, relative L2
GRAD_TOL = 1e-4   # dH/dp0, relative L2
COST_TOL = 1e-5   # H, relative
# Per-element bounds beside the relative L2 ones: the largest error of any
# single element, relative to the largest magnitude of the reference. A few
# wrong elements (a border row, a tile seam) that a whole-field norm could
# dilute fail these.
IMG_ELEM_TOL = 1e-4
GRAD_ELEM_TOL = 1e-3


def elem(a, b) -> float:
    """max |a - b| / max |b| (0 when b vanishes and a equals it)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = float(np.abs(b).max()) if b.size else 0.0
    d = float(np.abs(a - b).max()) if b.size else 0.0
    return d / mb if mb > 0 else d


def check_forward(plan, i, p, T):
    I_T, z_T, (H, data, reg) = oracle_forward(p, T)
    Ig, zg = host(plan.out_image[i]), host(plan.out_momentum[i])
    ri, rz = rel(Ig, I_T), rel(zg, z_T)
    ei, ez = elem(Ig, I_T), elem(zg, z_T)
    rH = abs(float(plan.out_cost[i, 0]) - H) / abs(H)
    announce(f"  forward pair {i}: image rel {ri:.2e} elem {ei:.2e}; momentum rel {rz:.2e} elem {ez:.2e}; "
             f"cost {rH:.2e}")
    assert ri <= IMG_TOL, ("image", ri)
    assert rz <= IMG_TOL or np.linalg.norm(z_T) == 0, ("momentum", rz)
    assert ei <= IMG_ELEM_TOL, ("image element", ei)
    assert ez <= IMG_ELEM_TOL or np.linalg.norm(z_T) == 0, ("momentum element", ez)
    assert rH <= COST_TOL, ("cost", rH)
    return ri, rz, rH


def check_grad(plan, i, p, T):
    H, g, data, reg = oracle_grad(p, T)
    return compare_grad(plan, i, H, g)


def compare_grad(plan, i, H, g):
    """Pair i of a plan against the oracle's cost H and gradient g."""
    gg = host(plan.out_grad[i])
    rg, eg = rel(gg, g), elem(gg, g)
    rH = abs(float(plan.out_cost[i, 0]) - H) / abs(H)
    announce(f"  grad pair {i}: rel {rg:.2e} elem {eg:.2e}; cost {rH:.2e}")
    assert rg <= GRAD_TOL, ("grad", rg)
    assert eg <= GRAD_ELEM_TOL, ("grad element", eg)
    assert rH <= COST_TOL, ("cost", rH)
    return rg, rH


def compare_adjoint_term(plan, i, pair, H, g, I_T):
    """Pair i against the oracle through the adjoint term of the gradient.

    dH/dp0 = zbar_0 + 2 lambda rho p0 (Eq. 4): at a momentum where descent
    has converged the two terms cancel, and the sum is rounding noise of both;
    the bound then applies to zbar_0, the adjoint's own output, taken from
    either gradient by subtracting the regulariser term in float64.

    zbar_0 is linear in the adjoint's seed, the residual R = I_T - J. A
    relative error e of the final image (bounded by IMG_TOL) is a relative
    error of up to e * kappa of R, kappa = |I_T| / |I_T - J| (the oracle's),
    which a good fit makes large; the bound on zbar_0 is therefore the larger
    of GRAD_TOL and IMG_TOL * kappa (the two stated tolerances chained through
    that linearity), and the element bound scales with it."""
    gg = host(plan.out_grad[i])
    reg = 2.0 * pair.lam * pair.rho * np.asarray(pair.p0, dtype=np.float64)
    zg, zo = gg - reg, np.asarray(g, dtype=np.float64) - reg
    rz, ez = rel(zg, zo), elem(zg, zo)
    rH = abs(float(plan.out_cost[i, 0]) - H) / abs(H)
    kappa = float(np.linalg.norm(I_T) / np.linalg.norm(np.asarray(I_T) - np.asarray(pair.target, dtype=np.float64)))
    tol = max(GRAD_TOL, IMG_TOL * kappa)
    etol = GRAD_ELEM_TOL * tol / GRAD_TOL
    announce(f"  adjoint term pair {i}: rel {rz:.2e} elem {ez:.2e} (|dH/dp0| / |zbar_0| = "
             f"{np.linalg.norm(g) / max(np.linalg.norm(zo), 1e-300):.2e}; kappa {kappa:.1f}, bound {tol:.2e}); "
             f"cost {rH:.2e}")
    assert rz <= tol, ("adjoint term", rz, tol)
    assert ez <= etol, ("adjoint term element", ez, etol)
    assert rH <= COST_TOL, ("cost", rH)
    return rz, rH
