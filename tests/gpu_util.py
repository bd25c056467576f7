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


def check_forward(plan, i, p, T):
    I_T, z_T, (H, data, reg) = oracle_forward(p, T)
    ri = rel(host(plan.out_image[i]), I_T)
    rz = rel(host(plan.out_momentum[i]), z_T)
    rH = abs(float(plan.out_cost[i, 0]) - H) / abs(H)
    assert ri <= IMG_TOL, ("image", ri)
    assert rz <= IMG_TOL or np.linalg.norm(z_T) == 0, ("momentum", rz)
    assert rH <= COST_TOL, ("cost", rH)
    return ri, rz, rH


def check_grad(plan, i, p, T):
    H, g, data, reg = oracle_grad(p, T)
    rg = rel(host(plan.out_grad[i]), g)
    rH = abs(float(plan.out_cost[i, 0]) - H) / abs(H)
    assert rg <= GRAD_TOL, ("grad", rg)
    assert rH <= COST_TOL, ("cost", rH)
    return rg, rH
