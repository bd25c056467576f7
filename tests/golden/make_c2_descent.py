"""Writes tests/golden/c2_descent.npz: the float64 oracle's gradient descent on
the single 240x240 brain-slice pair (T = 20, sigma = 5) from p0 = 0, 200
iterations at eta = 1 for each rho in {1.0, 0.5, 0.1} (Results: the costs are
minimised by gradient descent).

Stored per rho: the final momentum rounded to float32 (the "post-descent" p0
that the GPU parity tests feed to both the library and the oracle) and the
oracle's cost at the start of every iteration (the descent curve).

Only the oracle and the input recipes are used here. Run from the repository
root:  python tests/golden/make_c2_descent.py   (about 10 minutes of CPU,
three worker processes)."""
import os
import sys
from multiprocessing import get_context

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

RHOS = (1.0, 0.5, 0.1)
ITERS = 200
ETA = 1.0
OUT = os.path.join(ROOT, "tests", "golden", "c2_descent.npz")


def descend(rho):
    import oracle
    import synthetic

    p = synthetic.workload("c2", p0_kind="zero", rho=rho).pairs[0]
    p_final, hist = oracle.gradient_descent(p.source, p.target, p.p0, p.rho, p.sigma, p.lam, 20, iters=ITERS,
                                            eta=ETA)
    print(f"rho {rho}: cost {hist[0]:.6g} -> {hist[-1]:.6g}", flush=True)
    return rho, p_final.astype(np.float32), np.asarray(hist, dtype=np.float64)


def main():
    with get_context("fork").Pool(len(RHOS)) as pool:
        res = pool.map(descend, RHOS)
    out = {"rhos": np.asarray(RHOS), "iters": np.asarray(ITERS), "eta": np.asarray(ETA)}
    for rho, p, h in res:
        tag = f"{rho:.1f}".replace(".", "_")
        out[f"p0_rho{tag}"] = p
        out[f"cost_rho{tag}"] = h
    np.savez_compressed(OUT, **out)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
