"""Concurrent lanes: a batch split into lanes that run on their own streams
gives exactly the outputs of the single-lane plan, through captured graphs,
eager launches and the lockstep profiling mode, with and without admission
waves."""
import numpy as np
import pytest
import torch

import synthetic as G
from gpu_util import announce, host, specs
from paper_2106_08817_amd import SHOOT_LANES, SHOOT_NO_GRAPH, Plan

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _name(request):
    announce(request.node.nodeid)
    yield


def batch(ndim):
    if ndim == 2:
        shapes = [(40, 52), (67, 33), (96, 130), (30, 30), (75, 64), (52, 90), (33, 47)]
        sig = [2.0, 3.3, 5.0, 1.2, 2.5, 4.0, 1.8]
        T = 6
    else:
        shapes, sig, T = [(12, 17, 20), (9, 33, 14), (16, 16, 10)], [2.0, 1.5, 1.0], 4
    pairs = [G.small_pair(s, seed=900 + i, rho=0.2 + 0.1 * i, sigma=sig[i], p0_kind="realistic", lam=0.01)
             for i, s in enumerate(shapes)]
    return pairs, T


def outputs(plan, op):
    getattr(plan, op)()
    torch.cuda.synchronize()
    out = [host(plan.out_cost).copy()]
    for i in range(len(plan.out_image)):
        out += [host(plan.out_image[i]).copy(), host(plan.out_momentum[i]).copy()]
        if op == "grad":
            out.append(host(plan.out_grad[i]).copy())
    return out


def assert_same(a, b, what):
    assert len(a) == len(b)
    for k, (x, y) in enumerate(zip(a, b)):
        assert np.array_equal(x, y), f"{what}: output {k} differs (max |d| {np.max(np.abs(x - y))})"


@pytest.mark.parametrize("ndim", [2, 3])
def test_lanes_reproduce_the_single_lane_plan(ndim):
    pairs, T = batch(ndim)
    sp = specs(pairs)
    one = Plan(sp, T, SHOOT_LANES(1))
    assert one.lanes == 1
    ref = {op: outputs(one, op) for op in ("grad", "forward")}
    for k in ((2, 3, 4, 7) if ndim == 2 else (2, 3)):
        for flags, mode in ((0, "graph"), (SHOOT_NO_GRAPH, "eager")):
            announce(f"ndim {ndim} lanes {k} {mode}")
            plan = Plan(sp, T, SHOOT_LANES(k) | flags)
            assert plan.lanes == min(k, len(pairs))
            for op in ("grad", "forward", "grad"):  # replays after another op
                assert_same(outputs(plan, op), ref[op], f"{k} lanes, {mode}, {op}")
            plan.close()


def test_profiling_matches_and_counts_whole_batch_launches():
    pairs, T = batch(2)
    sp = specs(pairs)
    ref = outputs(Plan(sp, T, SHOOT_LANES(1)), "grad")
    stats = {}
    for k in (1, 4):
        plan = Plan(sp, T, SHOOT_LANES(k))
        plan.set_profiling(True)
        plan.reset_stats()
        assert_same(outputs(plan, "grad"), ref, f"profiled, {k} lanes")
        stats[k] = {name: n for name, (n, ms) in plan.kernel_stats().items()}
        plan.set_profiling(False)
        assert_same(outputs(plan, "grad"), ref, f"graph after profiling, {k} lanes")
    # a timed launch covers every lane: the counts do not grow with lanes
    assert stats[1] == stats[4]


def test_admission_waves_with_lanes():
    pairs, T = batch(2)
    sp = specs(pairs)
    ref = outputs(Plan(sp, T, SHOOT_LANES(1)), "grad")
    full = Plan(sp, T).workspace_bytes
    plan = Plan(sp, T, SHOOT_LANES(2), budget_bytes=int(0.6 * full))
    assert plan.waves >= 2 and plan.lanes == 2
    assert_same(outputs(plan, "grad"), ref, "waves of two lanes")


def test_calls_inside_the_callers_graph_capture():
    """Captured in the caller's own graph (the lanes then run one after
    another on the caller's stream); every replay, with eager work and
    synchronisation between replays, gives the eager outputs."""
    pairs, T = batch(2)
    sp = specs(pairs)
    ref = outputs(Plan(sp, T), "grad")
    plan = Plan(sp, T)
    assert plan.lanes == 3
    outputs(plan, "grad")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=s):
        plan.grad()
    for rep in range(3):
        announce(f"replay {rep}")
        plan.out_cost.fill_(-1.0)
        for t in plan.out_grad + plan.out_image + plan.out_momentum:
            t.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [host(plan.out_cost).copy()]
        for i in range(len(pairs)):
            got += [host(plan.out_image[i]).copy(), host(plan.out_momentum[i]).copy(), host(plan.out_grad[i]).copy()]
        assert_same(got, ref, f"replay {rep}")


def test_many_tiny_ragged_pairs():
    """150 pairs with extents from 2 to 40 (most smaller than one tile), in
    lanes and in budget waves: every pair's forward outputs equal its own
    single-pair plan's, its gradient agrees to 1e-6 (pairs moving 2 px or more
    per step take the adjoint's global-atomic scatter, whose summation order is
    not fixed), and sampled pairs match the oracle."""
    from gpu_util import check_grad, rel
    rng = np.random.default_rng(77)
    pairs = []
    for i in range(150):
        shape = (int(rng.integers(2, 41)), int(rng.integers(2, 41)))
        sigma = float(rng.uniform(0.5, 3.0))
        pairs.append(G.small_pair(shape, seed=1000 + i, rho=float(rng.uniform(0.0, 1.0)), sigma=sigma,
                                  p0_kind="realistic", lam=0.01))
    T = 3
    sp = specs(pairs)
    full = Plan(sp, T)
    assert full.lanes == 3
    full.grad()
    torch.cuda.synchronize()
    # the budget caps the whole workspace, every wave's header included: with
    # 150 tiny pairs the headers are most of it, so a budget just below the
    # single-wave plan's size is what forces waves here
    waves = Plan(sp, T, budget_bytes=full.workspace_bytes * 9 // 10)
    assert waves.waves >= 2
    waves.grad()
    torch.cuda.synchronize()
    for i in range(len(pairs)):
        one = Plan([sp[i]], T)
        one.grad()
        torch.cuda.synchronize()
        for plan in (full, waves):
            assert np.array_equal(host(plan.out_image[i]), host(one.out_image[0])), i
            assert np.array_equal(host(plan.out_momentum[i]), host(one.out_momentum[0])), i
            assert rel(host(plan.out_grad[i]), host(one.out_grad[0])) <= 1e-6, i
        one.close()
    for i in (0, 37, 99, 149):
        announce(f"tiny pair {i} shape {pairs[i].shape}")
        check_grad(full, i, pairs[i], T)


def test_many_tiny_ragged_volumes():
    """40 volumes with extents from 2 to 14 in 2 lanes: forward outputs equal
    the single-volume plans', gradients agree to 1e-6, sampled volumes match
    the oracle."""
    from gpu_util import check_grad, rel
    rng = np.random.default_rng(78)
    pairs = [G.small_pair(tuple(int(e) for e in rng.integers(2, 15, size=3)), seed=2000 + i,
                          rho=float(rng.uniform(0.0, 1.0)), sigma=float(rng.uniform(0.5, 2.0)),
                          p0_kind="realistic", lam=0.01) for i in range(40)]
    T = 2
    sp = specs(pairs)
    plan = Plan(sp, T)
    assert plan.lanes == 2
    plan.grad()
    torch.cuda.synchronize()
    for i in range(len(pairs)):
        one = Plan([sp[i]], T)
        one.grad()
        torch.cuda.synchronize()
        assert np.array_equal(host(plan.out_image[i]), host(one.out_image[0])), i
        assert rel(host(plan.out_grad[i]), host(one.out_grad[0])) <= 1e-6, i
        one.close()
    for i in (0, 13, 39):
        announce(f"tiny volume {i} shape {pairs[i].shape}")
        check_grad(plan, i, pairs[i], T)
