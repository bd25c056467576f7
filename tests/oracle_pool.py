"""CPU worker processes that run the float64 oracle for the full-size GPU
parity tests while the GPU tests run.

The pool is started when collection ends (tests/conftest.py), before any test
touches the GPU, so the workers are forks of a process without a device
context, and it is stopped when the session ends. Each job generates its own
inputs from the seeded recipes (the same arrays the test hands to the
library) and returns the oracle's results; nothing here reads any GPU output.
"""
import os
from multiprocessing import get_context

_pool = None
_pending = {}

WORKERS = 12


def _c3(i):
    import oracle
    import synthetic

    p = synthetic.workload_pair("c3", i)
    H, g, _, _ = oracle.cost_and_grad(p.source, p.target, p.p0, p.rho, p.sigma, p.lam, 20)
    return H, g


def _forward_and_grad(p, T):
    import oracle

    tr = oracle.shoot(p.source, p.p0, p.rho, p.sigma, T)
    I_T, z_T = tr.I[-1], tr.z[-1]
    D = oracle.max_displacement(tr, T)
    del tr
    H, g, _, _ = oracle.cost_and_grad(p.source, p.target, p.p0, p.rho, p.sigma, p.lam, T)
    return H, g, I_T, z_T, D


def _c4():
    import synthetic

    w = synthetic.workload("c4")
    return _forward_and_grad(w.pairs[0], w.T)


def _c5(i):
    import synthetic

    return _forward_and_grad(synthetic.workload_pair("c5", i), 15)


def _c2_post_descent(rho):
    import numpy as np

    import synthetic
    from golden_fixtures import c2_post_descent_p0

    p = synthetic.workload("c2", p0_kind="zero", rho=rho).pairs[0]
    p.p0 = np.ascontiguousarray(c2_post_descent_p0(rho))
    return _forward_and_grad(p, 20)


def jobs():
    """(key, function, args) of every job, longest first."""
    import synthetic

    out = [(("c4",), _c4, ())]
    classes = sorted(synthetic.c5_shape_classes().items(), key=lambda kv: -kv[0][0] * kv[0][1] * kv[0][2])
    out += [(("c5", i), _c5, (i,)) for _, i in classes]
    out += [(("c2", rho), _c2_post_descent, (rho,)) for rho in (1.0, 0.5, 0.1)]
    out += [(("c3", i), _c3, (i,)) for i in range(64)]
    return out


def start():
    global _pool
    if _pool is not None:
        return
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    _pool = get_context("fork").Pool(WORKERS)
    for key, fn, args in jobs():
        _pending[key] = _pool.apply_async(fn, args)


def started() -> bool:
    return _pool is not None


def result(key, timeout=900):
    """The oracle's result for `key`, waited for with a progress line every
    30 s (a wait of minutes on a large volume is not a hang)."""
    import sys
    import time
    from multiprocessing import TimeoutError as PoolTimeout

    if _pool is None:
        raise RuntimeError("the oracle pool was not started at collection")
    t0 = time.monotonic()
    while True:
        left = timeout - (time.monotonic() - t0)
        if left <= 0:
            raise PoolTimeout(f"oracle job {key} not done after {timeout} s")
        try:
            return _pending[key].get(min(30.0, left))
        except PoolTimeout:
            sys.__stderr__.write(f"[gpu-case]   waiting for the oracle's {key} ({time.monotonic() - t0:.0f} s)\n")
            sys.__stderr__.flush()


def stop():
    global _pool
    if _pool is not None:
        _pool.terminate()
        _pool.join()
        _pool = None
        _pending.clear()
