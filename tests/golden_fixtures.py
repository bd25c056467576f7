"""Readers of the fixtures under tests/golden/ (values the paper prints, each
file citing where)."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_values(name: str) -> dict:
    """key = value lines of a fixture; '#' starts a comment."""
    out = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                out[k.strip()] = float(v) if "." in v else int(v)
    return out


def fig1_steps() -> tuple:
    """(Eulerian steps, semi-Lagrangian steps) of the paper's Fig. 1."""
    v = read_values("fig1_time_steps.txt")
    return v["eulerian_steps"], v["semi_lagrangian_steps"]


def c2_descent() -> dict:
    """The float64 oracle's 200-iteration gradient descent on the 240x240 pair
    (written by tests/golden/make_c2_descent.py, which calls only the oracle):
    {rho: (final p0 as float32, cost at the start of every iteration)}."""
    import numpy as np

    with np.load(os.path.join(GOLDEN, "c2_descent.npz"), allow_pickle=False) as z:
        out = {}
        for rho in z["rhos"]:
            tag = f"{float(rho):.1f}".replace(".", "_")
            out[float(rho)] = (z[f"p0_rho{tag}"], z[f"cost_rho{tag}"])
    return out


def c2_post_descent_p0(rho: float):
    return c2_descent()[float(rho)][0]
