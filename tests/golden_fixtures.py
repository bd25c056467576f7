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
