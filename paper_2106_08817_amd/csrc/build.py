"""Builds libshoot.so (gfx950) in-tree with hipcc: every source is compiled to
an object in parallel (objects under _build/ at the repository root), then the
objects are linked into the shared library."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
SOURCES = ["kernels.hip", "kernels_adj3.hip", "kernels_mfma.hip", "kernels_unfused.hip", "kernels_opt.hip", "shoot_api.cpp", "lbfgs_api.cpp", "tune_cache.cpp"]
OUT = os.path.join(PKG, "libshoot.so")
OBJ_DIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # keep packed FP32 instructions out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-function",
    "-fvisibility=hidden",
]


def _quiet(stderr: str) -> str:
    # the host pass does not know the packed-fp32 feature and says so; drop that noise
    return "\n".join(l for l in stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = _quiet(res.stderr)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}): {' '.join(cmd)}\n{err}")
    if err and verbose:
        print(err, file=sys.stderr)


def build(verbose: bool = True) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", HERE]
    objs, cmds = [], []
    for s in SOURCES:
        o = os.path.join(OBJ_DIR, os.path.splitext(s)[0] + ".o")
        objs.append(o)
        cmds.append([HIPCC] + FLAGS + inc + ["-c", "-x", "hip", os.path.join(HERE, s), "-o", o])
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, c, verbose) for c in cmds]:
            f.result()
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", OUT + ".tmp"], verbose)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build()
