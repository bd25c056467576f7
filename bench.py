#!/usr/bin/env python3
"""Throughput of batched cost + dH/dp0 evaluations (forward shooting, cost,
hand-written discrete adjoint with sqrt(T) checkpointing) on one MI355X.

A step is one cost + gradient evaluation of every pair of the workload (by
default the 16 ragged 3-D volumes), replayed from the plan's captured HIP
graphs, with all inputs resident in HBM. The JSON line reports:

* value: voxel-steps/s = sum_i N_i * T per evaluation / seconds (a step of the
  scheme counts once per evaluation, although forward, recompute and adjoint
  all visit it); pair_evals_per_s alongside;
* unfused: the same evaluations through the per-pair, one-kernel-per-primitive
  path of the same library, and the speed-up over it;
* roofline: the kernel family with the largest share of the step time, its
  algorithmic bytes per launch over its average launch duration (HIP events
  around its launches on the stream they run on), against 8 TB/s, beside the
  library's own streaming copy of the same bytes;
* cpu_baseline: the float64 oracle on the host, on a bounded sample;
* extra: the other workloads (the 64-pair 2-D batch, the single 3-D volume,
  the single 2-D pair), the device gradient descent of the 2-D pair and the
  throughput at its final momentum, the large-step regime (adjoint fallback
  paths), full storage, deformation map, L-BFGS and the integration options.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "cost+grad evals/sec & voxel-steps/s, batched adjoint vs per-pair unfused, %HBM"
HBM_PEAK_GBPS = 8000.0

WORKLOADS = {
    "c3": "64 ragged 2-D brain-slice pairs, H, W iid in {96,128,192,240,320}, sigma_i ~ U[2,6], "
          "rho_i ~ U[0.05,1], T=20, cost+grad",
    "c2": "one 2-D 240x240 brain-slice pair, sigma=5, rho=0.5, T=20, cost+grad",
    "c4": "one 3-D 160x192x160 brain-volume pair, sigma=4, rho=0.3, T=15, cost+grad",
    "c5": "16 ragged 3-D brain volumes from {96^3, 128^3, 128x160x128, 160x192x160}, sigma=4, "
          "rho_i ~ U[0.1,1], T=15, cost+grad",
}

# Algorithmic (compulsory) bytes per voxel of one launch of each kernel family:
# float32 fields each kernel must read and write once, d = 2 or 3.
def bytes_per_voxel(name: str, d: int) -> int:
    f = 4
    table = {
        "xpass_gradmul": 2 + d,          # read I, z; write d channels
        "xpass_plain": 2 * d,            # read d, write d
        "spass_mid": 2 * d,
        "spass_v": 2 * d,
        "spass_mbar": 2 * d,
        "advect": d + 2 + 2,             # read v, I, z; write I', z'
        "advect_adjoint": (d + 2 + 2) + (2 + d),  # read v, I, z, Ibar', zbar'; write Interp^T parts, vbar
        "epilogue": (d + 2 + 2) + 2,     # read mbar, I, z, Interp^T parts; write Ibar, zbar
        "init": 4,
        "deform": 3 * d,                 # read v, psi; write psi
        "descend": 3,                    # read p0, dH/dp0; write p0
        "fill": 0,
        "finalize": 0,
    }
    return f * table.get(name, 0)


# rocprofv3 kernel names -> kernel families of the profiling statistics
def family_of(kernel_name: str) -> str:
    n = kernel_name
    if "k_adv_adj" in n:
        return "advect_adjoint"
    if "k_advect" in n:
        return "advect"
    if "k_epilogue" in n:
        return "epilogue"
    if "k_xpass" in n:
        return "xpass_gradmul" if "true>" in n else "xpass_plain"
    if "k_spass" in n:
        mode = n.split("k_spass<")[1].split(">")[0].split(",")[2].strip()
        return {"0": "spass_mid", "1": "spass_v", "2": "spass_mbar"}[mode]
    if "k_init" in n:
        return "init"
    if "k_deform" in n:
        return "deform"
    if "k_descend" in n:
        return "descend"
    if "k_finalize" in n:
        return "finalize"
    if "k_fill_u32" in n:
        return "fill"
    return n


def kernel_source_sha() -> str:
    """Hash of every device source and header of the library (the kernels'
    code), in name order."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2106_08817_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(name.encode())
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str, launches_ref: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = rec.get(workload, {}).get(kernel)
    if not entry or entry.get("source_sha") != kernel_source_sha():
        return None
    return entry.get("bytes_per_launch")


def copy_probe(mbytes: int, reps: int) -> None:
    """The library's streaming copy of known size, for calibrating the
    FETCH_SIZE / WRITE_SIZE counters (run under rocprofv3 --pmc)."""
    import torch

    from paper_2106_08817_amd import api

    n = mbytes * (1 << 20) // 4
    a = torch.rand(n, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(reps):
        api.stream_copy(a, b)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "reps": reps}))


def write_traffic(workload: str, fetch_csv: str, write_csv: str, copy_fetch_csv: str, copy_write_csv: str,
                  copy_bytes: int, path: str) -> None:
    """Per-launch HBM traffic of every kernel family from two rocprofv3 --pmc
    runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what
    the same counter reads for a plain copy of known size; written to
    profiles/traffic.json with the hash of the kernel sources."""
    import csv
    from collections import defaultdict

    def per_kernel(path, counter):
        acc = defaultdict(list)
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] == counter:
                    acc[row["Kernel_Name"]].append(float(row["Counter_Value"]))
        return acc

    def copy_kib(path, counter):
        vals = [v for k, vs in per_kernel(path, counter).items() for v in vs if "k_stream_copy" in k]
        return sorted(vals)[len(vals) // 2]

    f_scale = copy_bytes / (1024.0 * copy_kib(copy_fetch_csv, "FETCH_SIZE"))
    w_scale = copy_bytes / (1024.0 * copy_kib(copy_write_csv, "WRITE_SIZE"))
    fetch = per_kernel(fetch_csv, "FETCH_SIZE")
    write = per_kernel(write_csv, "WRITE_SIZE")
    fam = defaultdict(lambda: {"fetch": [], "write": []})
    for k, vs in fetch.items():
        if "shoot::" in k and "k_stream_copy" not in k:
            fam[family_of(k)]["fetch"] += vs
    for k, vs in write.items():
        if "shoot::" in k and "k_stream_copy" not in k:
            fam[family_of(k)]["write"] += vs
    rec = {}
    if os.path.exists(path):
        with open(path) as fh:
            rec = json.load(fh)
    sha = kernel_source_sha()
    out = {}
    for name, d in fam.items():
        if not d["fetch"] or not d["write"]:
            continue
        fb = 1024.0 * f_scale * sum(d["fetch"]) / len(d["fetch"])
        wb = 1024.0 * w_scale * sum(d["write"]) / len(d["write"])
        out[name] = {"bytes_per_launch": fb + wb, "fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                     "dispatches": len(d["fetch"]), "source_sha": sha}
    rec[workload] = out
    rec["_calibration"] = {"copy_bytes": copy_bytes, "fetch_scale": f_scale, "write_scale": w_scale}
    with open(path, "w") as fh:
        json.dump(rec, fh, indent=1, sort_keys=True)
    print(json.dumps(out, indent=1))


def build_plan(workload, flags, torch, api):
    specs = []
    for p in workload.pairs:
        t = lambda a: torch.from_numpy(a).to("cuda:0")  # noqa: E731
        specs.append(api.PairSpec(t(p.source), t(p.p0), p.rho, p.sigma, p.lam, t(p.target)))
    return api.Plan(specs, workload.T, flags, outputs=("grad", "cost"))


def time_evals(plan, n, torch):
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(n):
        plan.grad()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1000.0


def per_eval_ms(plan, n, torch):
    """Median and minimum of n individually timed evaluations (events on the
    stream around each graph replay)."""
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(n + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(n):
        plan.grad()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    ms = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(n))
    return ms[n // 2], ms[0]


def _oracle_eval(args):
    import oracle
    t0 = time.perf_counter()
    oracle.cost_and_grad(*args)
    return time.perf_counter() - t0


def cpu_baseline(workload, seconds, workers):
    """2-D workloads: the oracle as it stands on the host, single-threaded
    NumPy on the first pairs of the workload until about `seconds` of work (at
    least one pair), then the same pairs spread over `workers` processes (one
    pair at a time each) for the aggregate rate of that many cores. Runs before
    anything touches the GPU, so that the worker processes fork from a process
    without a device context."""
    import multiprocessing as mp

    vs, used, done = 0, 0.0, 0
    for p in workload.pairs:
        used += _oracle_eval((p.source, p.target, p.p0, p.rho, p.sigma, p.lam, workload.T))
        vs += p.size * workload.T
        done += 1
        if used >= seconds:
            break
    single = {"value": vs / used, "unit": "voxel-steps/s", "cores": 1,
              "sample": f"first {done} of {len(workload.pairs)} pairs, one float64 cost+grad evaluation each "
                        f"({used:.1f} s, single-threaded NumPy)"}
    jobs = [(p.source, p.target, p.p0, p.rho, p.sigma, p.lam, workload.T) for p in workload.pairs[:done]]
    with mp.get_context("fork").Pool(workers) as pool:
        t0 = time.perf_counter()
        cpu_s = sum(pool.map(_oracle_eval, jobs, chunksize=1))
        wall = time.perf_counter() - t0
    return {"value": vs / wall, "unit": "voxel-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"the same {done} pairs spread over {workers} worker processes, one float64 cost+grad "
                      f"evaluation each ({wall:.1f} s wall, {cpu_s:.1f} s of CPU work, single-threaded NumPy "
                      "per process)",
            "single_core": single}


def cpu_baseline_3d(workload, t_sample, workers):
    """3-D workloads, where one float64 oracle evaluation of a volume at full T
    takes minutes: every evaluation is cost + gradient at t_sample steps (the
    oracle stores the whole trajectory, so its time per step does not depend on
    T). Single core: the first volume of each shape class, one process per class
    (single-threaded NumPy each, run side by side), extrapolated to the whole
    batch at its T. All cores: `workers` processes evaluating the batch's first
    volume of the smallest shape class at once, for the aggregate rate of that
    many cores. Runs before anything touches the GPU."""
    import multiprocessing as mp

    classes = {}
    for i, p in enumerate(workload.pairs):
        classes.setdefault(p.shape, i)
    jobs = [(workload.pairs[i].source, workload.pairs[i].target, workload.pairs[i].p0, workload.pairs[i].rho,
             workload.pairs[i].sigma, workload.pairs[i].lam, t_sample) for i in classes.values()]
    with mp.get_context("fork").Pool(len(jobs)) as pool:
        secs = pool.map(_oracle_eval, jobs, chunksize=1)
    per_step = {shp: s / t_sample for shp, s in zip(classes, secs)}  # seconds per step of one volume
    batch_s = sum(per_step[p.shape] for p in workload.pairs) * workload.T
    vs = workload.voxel_steps
    single = {"value": vs / batch_s, "unit": "voxel-steps/s", "cores": 1,
              "sample": f"one float64 cost+grad evaluation at T={t_sample} of the first volume of each of the "
                        f"{len(classes)} shape classes ({sum(secs):.1f} s of CPU work, single-threaded NumPy, one "
                        f"process per class side by side), extrapolated to the {len(workload.pairs)} volumes at "
                        f"T={workload.T}: {batch_s:.0f} s per batch evaluation",
              "seconds_per_step": {"x".join(map(str, k)): v for k, v in per_step.items()}}
    small = min(classes, key=lambda shp: shp[0] * shp[1] * shp[2])
    q = workload.pairs[classes[small]]
    with mp.get_context("fork").Pool(workers) as pool:
        t0 = time.perf_counter()
        cpu_s = sum(pool.map(_oracle_eval, [(q.source, q.target, q.p0, q.rho, q.sigma, q.lam, t_sample)] * workers,
                             chunksize=1))
        wall = time.perf_counter() - t0
    return {"value": workers * q.size * t_sample / wall, "unit": "voxel-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} worker processes each evaluating cost+grad of the batch's first "
                      f"{'x'.join(map(str, small))} volume at T={t_sample} at once ({wall:.1f} s wall, "
                      f"{cpu_s:.1f} s of CPU work, single-threaded NumPy per process)",
            "single_core": single}


def copy_rate(nbytes: int, torch, api, reps: int = 20) -> float:
    """GB/s of the library's streaming copy kernel reading and writing nbytes
    in total (the bandwidth a kernel that touches every byte once reaches at
    this working-set size)."""
    n = max(4, (nbytes // 8) // 4 * 4)
    a = torch.rand(n, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        api.stream_copy(a, b)
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        api.stream_copy(a, b)
    e1.record(stream)
    torch.cuda.synchronize()
    assert torch.equal(a, b), "stream copy mismatch"
    return 8.0 * n * reps / (e0.elapsed_time(e1) / 1000.0) / 1e9


def scheme_comparison(wl, steps, warmup, torch, api, synthetic):
    """The integration options the paper compares: shoot_forward time over the
    workload for each, and the stability rerun (rho = 0 shot of a disk toward a
    'C': range overshoot of I_T and total variation of z_T; the Eulerian
    scheme at dt = 1/38, the semi-Lagrangian ones at 1/20)."""
    def specs_of(pairs):
        return [api.PairSpec(torch.from_numpy(p.source).cuda(), torch.from_numpy(p.p0).cuda(), p.rho, p.sigma,
                             p.lam, torch.from_numpy(p.target).cuda()) for p in pairs]

    out = {}
    flags = {"semi_lagrangian": 0, "eulerian": api.SHOOT_SCHEME_EULERIAN, "mixed": api.SHOOT_SCHEME_MIXED}
    for name, f in flags.items():
        plan = api.Plan(specs_of(wl.pairs), wl.T, f, outputs=("image", "momentum", "cost"))
        for _ in range(warmup):
            plan.forward()
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            plan.forward()
        e1.record(stream)
        torch.cuda.synchronize()
        out[name] = {"forward_ms": e0.elapsed_time(e1) / steps}
        plan.close()
    S, J, p0 = synthetic.ripple_case()
    lo, hi = float(S.min()), float(S.max())
    for name, f, T in (("semi_lagrangian", 0, 20), ("eulerian", api.SHOOT_SCHEME_EULERIAN, 38),
                       ("mixed", api.SHOOT_SCHEME_MIXED, 20)):
        t = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
        plan = api.Plan([api.PairSpec(t(S), t(p0), 0.0, 3.0, 0.01, t(J))], T, f, outputs=("image", "momentum"))
        plan.forward()
        torch.cuda.synchronize()
        I = plan.out_image[0].double()
        z = plan.out_momentum[0].double()
        over = max(float(I.max()) - hi, lo - float(I.min()), 0.0)
        tv = float(sum(z.diff(dim=a).abs().sum() for a in range(z.dim())))
        out[name].update({"ripple_case_T": T, "ripple_case_overshoot": over, "ripple_case_z_total_variation": tv})
        plan.close()
    return out


def lbfgs_rate(wl, iters, torch, api):
    """Wall time of batched L-BFGS iterations over the workload (every pair at
    once; each iteration evaluates cost + gradient once per line-search trial
    and synchronises for the per-pair step decisions)."""
    specs = [api.PairSpec(torch.from_numpy(p.source).cuda(), torch.from_numpy(p.p0).cuda(), p.rho, p.sigma,
                          p.lam, torch.from_numpy(p.target).cuda()) for p in wl.pairs]
    plan = api.Plan(specs, wl.T, 0, outputs=("grad", "cost"))
    opt = api.LBFGS(plan)
    c0, _ = opt.step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evals = 0
    for _ in range(iters):
        c, e = opt.step()
        evals += e
    secs = time.perf_counter() - t0
    cost_now = plan.out_cost[:, 0].double().sum().item()
    opt.close()
    plan.close()
    return {"ms_per_iteration": 1000.0 * secs / iters, "evaluations_per_iteration": evals / iters,
            "summed_cost_first": float(sum(c0)), "summed_cost_after": cost_now, "iterations": iters + 1}


def forward_deformation(wl, steps, warmup, torch, api):
    """shoot_forward over the workload with and without the deformation map
    psi_T, and the deformation kernel's launch duration and bandwidth."""
    def plan_for(outs, flags=0):
        specs = [api.PairSpec(torch.from_numpy(p.source).cuda(), torch.from_numpy(p.p0).cuda(), p.rho, p.sigma,
                              p.lam, torch.from_numpy(p.target).cuda()) for p in wl.pairs]
        return api.Plan(specs, wl.T, flags, outputs=outs)

    def timed(plan):
        for _ in range(warmup):
            plan.forward()
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            plan.forward()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    d = wl.pairs[0].ndim
    voxels = sum(p.size for p in wl.pairs)
    base = plan_for(("image", "momentum", "cost"))
    ms0 = timed(base)
    base.close()
    plan = plan_for(("image", "momentum", "cost", "deformation"))
    ms1 = timed(plan)
    plan.close()
    # the kernel's duration as one launch over the whole batch (one lane)
    plan = plan_for(("image", "momentum", "cost", "deformation"), api.SHOOT_LANES(1))
    plan.forward()
    plan.set_profiling(True)
    plan.reset_stats()
    plan.forward()
    n, ms = plan.kernel_stats()["deform"]
    plan.close()
    avg_us = 1000.0 * ms / n
    return {"forward_ms": ms0, "forward_with_deformation_ms": ms1, "deform_launches": n,
            "deform_avg_us": avg_us,
            "deform_algorithmic_GBps": bytes_per_voxel("deform", d) * voxels / (avg_us * 1e-6) / 1e9,
            "note": "psi_T: psi_0 = Id, psi_{t+1} = psi_t o (Id - dt v_t), one extra kernel per forward step"}


def kernel_profile(wl, flags, tuning, profile_steps, torch, api):
    """Per-kernel launch durations (HIP events around every launch on its
    stream, the library's profiling mode) on a one-lane plan of the workload,
    so that each launch covers every pair (the timed plan's lanes split every
    kernel into concurrent launches)."""
    d = wl.pairs[0].ndim
    voxels = sum(p.size for p in wl.pairs)
    pplan = build_plan(wl, flags | api.SHOOT_LANES(1), torch, api)
    if tuning is not None:
        pplan.tuning = tuning
    pplan.grad()
    pplan.set_profiling(True)
    pplan.reset_stats()
    for _ in range(profile_steps):
        pplan.grad()
    stats = pplan.kernel_stats()
    pplan.close()
    kernels = {}
    for kname, (n, ms) in stats.items():
        if n == 0:
            continue
        bpl = bytes_per_voxel(kname, d) * voxels
        avg = ms / n
        kernels[kname] = {"launches_per_eval": n / profile_steps, "avg_us": 1000.0 * avg,
                          "ms_per_eval": ms / profile_steps,
                          "algorithmic_GBps": (bpl / (avg / 1000.0)) / 1e9 if avg > 0 else None}
    return kernels


def measure(wl, label, steps, warmup, profile_steps, flags, autotune, torch, api, keep_plan=False, fixed=None,
            unfused_steps=0):
    """Times `steps` graph replays of cost + dH/dp0 over workload wl, then one
    profiled pass for per-kernel durations and the roofline record; with
    unfused_steps > 0 also the per-pair unfused path of the same library."""
    d = wl.pairs[0].ndim
    voxels = sum(p.size for p in wl.pairs)
    vsteps = voxels * wl.T
    plan = build_plan(wl, flags, torch, api)
    tuning = None
    if fixed is not None:
        plan.tuning = fixed
        tuning = plan.tuning
    elif autotune:
        t_tune = time.perf_counter()
        tuning = plan.autotune()
        print(f"[bench] {label} autotune: choices {tuning} ({time.perf_counter() - t_tune:.1f} s)", file=sys.stderr,
              flush=True)
    for _ in range(warmup):
        plan.grad()
    torch.cuda.synchronize()
    secs = time_evals(plan, steps, torch)
    ms_per_step = 1000.0 * secs / steps
    ms_median, ms_min = per_eval_ms(plan, min(max(steps, 1), 20), torch)
    value = vsteps * steps / secs
    costs = plan.out_cost[:, 0].cpu().numpy()
    assert np.all(np.isfinite(costs)), "non-finite cost"
    disp = plan.displacements()
    print(f"[bench] {label} fused: {ms_per_step:.3f} ms/eval, {value:.4g} voxel-steps/s", file=sys.stderr, flush=True)

    kernels = kernel_profile(wl, flags, plan.tuning, profile_steps, torch, api)
    dom = max(kernels, key=lambda k: kernels[k]["ms_per_eval"])
    dk = kernels[dom]
    bpl = bytes_per_voxel(dom, d) * voxels
    achieved = bpl / (dk["avg_us"] * 1e-6) / 1e9
    copy_gbps = copy_rate(bpl, torch, api)
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS, "traffic": measured_traffic(dom, wl.name, None),
                "algorithmic_bytes_per_launch": bpl, "avg_launch_us": dk["avg_us"],
                "copy_same_bytes_GBps": copy_gbps, "frac_of_copy": achieved / copy_gbps,
                "launch": "one launch over the whole batch (a one-lane plan of the same pairs and tuning)"}
    step_bytes = sum(bytes_per_voxel(k, d) * voxels * v["launches_per_eval"] for k, v in kernels.items())
    print(f"[bench] {label} dominant kernel {dom}: {dk['avg_us']:.1f} us/launch, {achieved:.0f} GB/s algorithmic "
          f"(the library's streaming copy of the same bytes: {copy_gbps:.0f} GB/s)", file=sys.stderr, flush=True)
    bound = 2.0 if d == 2 else 1.0
    out = {"pairs": len(wl.pairs), "voxels": voxels, "T": wl.T, "voxel_steps": vsteps, "value": value,
           "unit": "voxel-steps/s", "ms_per_eval": ms_per_step, "secs": secs,
           "pair_evals_per_s": len(wl.pairs) * steps / secs, "steps": steps, "tuning": tuning,
           "lanes": plan.lanes, "ms_per_eval_median": ms_median, "ms_per_eval_min": ms_min,
           "step_algorithmic_GBps": step_bytes / (ms_per_step / 1000.0) / 1e9,
           "step_hbm_frac": step_bytes / (ms_per_step / 1000.0) / 1e9 / HBM_PEAK_GBPS,
           "step_bytes": step_bytes, "roofline": roofline, "kernels": kernels,
           "step_displacement_px": {"p5": float(np.percentile(disp, 5)), "median": float(np.median(disp)),
                                    "p95": float(np.percentile(disp, 95)), "max": float(disp.max()),
                                    "share_of_steps_on_gather_path": float(np.mean(disp < bound))}}
    if unfused_steps > 0:
        uplan = build_plan(wl, api.SHOOT_UNFUSED, torch, api)
        uplan.grad()
        torch.cuda.synchronize()
        usecs = time_evals(uplan, unfused_steps, torch)
        uval = vsteps * unfused_steps / usecs
        ucosts = uplan.out_cost[:, 0].cpu().numpy().astype(np.float64)
        out["unfused"] = {"value": uval, "unit": "voxel-steps/s", "ms_per_eval": 1000.0 * usecs / unfused_steps,
                          "speedup": value / uval, "steps": unfused_steps,
                          "path": "same library, per pair in sequence, one kernel per primitive, full trajectory "
                                  "stored, global-atomic scatter, no graph",
                          "max_rel_cost_diff": float(np.max(np.abs(ucosts - costs) / np.abs(costs)))}
        uplan.close()
        print(f"[bench] {label} unfused: {out['unfused']['ms_per_eval']:.1f} ms/eval, speed-up "
              f"{out['unfused']['speedup']:.1f}x", file=sys.stderr, flush=True)
    if keep_plan:
        out["_plan"] = plan
    else:
        plan.close()
    return out


def descent_c2(w2_of_rho, iters, eval_steps, torch, api):
    """Device gradient descent (shoot_descend: eta = 1, halved per pair when
    its cost rises) on the 240x240 pair from p0 = 0 for each rho, the cost at
    every iteration, and the evaluation rate at the momentum it reaches."""
    out = {}
    for rho, w in w2_of_rho.items():
        p = w.pairs[0]
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")  # noqa: E731
        p0 = t(np.zeros_like(p.p0))
        plan = api.Plan([api.PairSpec(t(p.source), p0, p.rho, p.sigma, p.lam, t(p.target))], w.T, 0,
                        outputs=("grad", "cost"))
        costs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(iters):
            plan.descend(1.0, reset=(it == 0))
            costs.append(float(plan.out_cost[0, 0]))  # the cost at the p0 of this iteration
        secs = time.perf_counter() - t0
        # the momentum now in p0 is the descent's result: evaluate there
        for _ in range(3):
            plan.grad()
        ev = time_evals(plan, eval_steps, torch)
        disp = plan.displacements()
        out[f"rho_{rho}"] = {"cost_first": costs[0], "cost_last": costs[-1],
                             "cost_every_10": costs[::10] + [costs[-1]],
                             "ms_per_iteration": 1000.0 * secs / iters,
                             "post_descent_ms_per_eval": 1000.0 * ev / eval_steps,
                             "post_descent_voxel_steps_per_s": w.voxel_steps * eval_steps / ev,
                             "post_descent_max_step_px": float(disp.max())}
        print(f"[bench] c2 descent rho {rho}: cost {costs[0]:.5g} -> {costs[-1]:.5g} in {iters} iterations "
              f"({1000.0 * secs / iters:.2f} ms each, with a cost read-back)", file=sys.stderr, flush=True)
        plan.close()
    return out


def strip(r):
    for key in ("secs", "step_bytes", "_plan"):
        r.pop(key, None)
    return r


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--profile-steps", type=int, default=2, help="evaluations timed per kernel")
    ap.add_argument("--unfused-steps", type=int, default=1)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="2-D: single-core oracle sample length")
    ap.add_argument("--cpu-steps-3d", type=int, default=2, help="3-D: steps of each oracle sample evaluation")
    ap.add_argument("--no-unfused", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--flags", type=int, default=0, help="extra plan flags (bit mask of SHOOT_*)")
    ap.add_argument("--no-extra", action="store_true", help="only the headline workload")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shapes")
    ap.add_argument("--tuning", default=None, metavar="C0,C1,...",
                    help="launch-shape choices to use instead of autotuning (comma-separated 0/1)")
    ap.add_argument("--descent-iters", type=int, default=200)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MB",
                    help="only run the library's streaming copy of MB MiB (counter calibration) and exit")
    ap.add_argument("--write-traffic", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="only turn rocprofv3 counter CSVs into profiles/traffic.json and exit")
    ap.add_argument("--copy-mb", type=int, default=1024, help="size of the calibration copy (MiB)")
    ap.add_argument("--traffic-out", default=os.path.join(ROOT, "profiles", "traffic.json"))
    args = ap.parse_args()

    if args.copy_probe:
        copy_probe(args.copy_probe, 5)
        return
    if args.write_traffic:
        write_traffic(args.workload, *args.write_traffic, args.copy_mb * (1 << 20), args.traffic_out)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE={world}): the pairs of a "
              "batch are independent, and the benchmark measures one GPU's share of such a batch.", file=sys.stderr)
        sys.exit(2)

    import synthetic

    t_gen = time.perf_counter()
    wl = synthetic.workload(args.workload, p0_kind="realistic")
    print(f"[bench] {args.workload}: {len(wl.pairs)} pairs, {sum(p.size for p in wl.pairs)} voxels, T={wl.T} "
          f"(inputs {time.perf_counter() - t_gen:.1f} s)", file=sys.stderr, flush=True)

    # the oracle's CPU baseline first, before anything touches the GPU
    cpu = None
    if not args.no_cpu_baseline:
        workers = max(1, min(16, os.cpu_count() or 1))
        t_cpu = time.perf_counter()
        if wl.pairs[0].ndim == 3:
            cpu = cpu_baseline_3d(wl, args.cpu_steps_3d, workers)
        else:
            cpu = cpu_baseline(wl, args.cpu_seconds, workers)
        print(f"[bench] cpu baseline: {cpu['value']:.4g} voxel-steps/s on {workers} cores, "
              f"{cpu['single_core']['value']:.4g} on one ({time.perf_counter() - t_cpu:.0f} s)", file=sys.stderr,
              flush=True)

    import torch

    from paper_2106_08817_amd import api

    fixed = [int(c) for c in args.tuning.split(",")] if args.tuning else None
    main_run = measure(wl, args.workload, args.steps, args.warmup, args.profile_steps, args.flags,
                       not args.no_autotune and fixed is None, torch, api, keep_plan=True, fixed=fixed,
                       unfused_steps=0 if args.no_unfused else args.unfused_steps)
    plan = main_run.pop("_plan")
    voxels, value = main_run["voxels"], main_run["value"]
    tuning = main_run["tuning"]
    plan.close()

    extra = {}
    if not args.no_extra:
        autotune = not args.no_autotune
        # the same batch with every state stored (no recomputation)
        fplan = build_plan(wl, api.SHOOT_FULL_STORE | args.flags, torch, api)
        if tuning is not None:
            fplan.tuning = tuning
        for _ in range(args.warmup):
            fplan.grad()
        fsecs = time_evals(fplan, args.steps, torch)
        extra["full_store"] = {"value": wl.voxel_steps * args.steps / fsecs, "unit": "voxel-steps/s",
                               "ms_per_eval": 1000.0 * fsecs / args.steps,
                               "note": "all T states kept (no recomputation); same kernels"}
        fplan.close()
        # the other workloads, each with its own roofline record
        others = {"c5": "batched_3d_c5", "c4": "single_volume_c4", "c3": "batched_2d_c3"}
        for name, key in others.items():
            if name == args.workload:
                continue
            t_gen = time.perf_counter()
            w = synthetic.workload(name, p0_kind="realistic")
            print(f"[bench] {name}: inputs {time.perf_counter() - t_gen:.1f} s", file=sys.stderr, flush=True)
            r = measure(w, name, args.steps, args.warmup, 1, args.flags, autotune, torch, api,
                        unfused_steps=0 if (args.no_unfused or name == "c5") else args.unfused_steps)
            r["workload"] = f"{name}: {WORKLOADS[name]}"
            extra[key] = strip(r)
            # the large-step regime of the batches: the adjoint's fallback paths
            if name in ("c3", "c5"):
                ls = synthetic.large_step(w)
                r = measure(ls, name + " large-step", args.steps, args.warmup, 1, args.flags, autotune, torch, api)
                r["workload"] = (f"{name} images, realistic momentum x {synthetic.LARGE_STEP_SCALE:g}, rho = 0, "
                                 f"T = {ls.T}: feet move ~1-3 {'px' if name == 'c3' else 'voxels'} per step")
                extra[key + "_large_step"] = strip(r)
        if args.workload in ("c5",):
            ls = synthetic.large_step(wl)
            r = measure(ls, "c5 large-step", args.steps, args.warmup, 1, args.flags, autotune, torch, api)
            r["workload"] = (f"c5 images, realistic momentum x {synthetic.LARGE_STEP_SCALE:g}, rho = 0, T = {ls.T}: "
                             "feet move ~1-2.5 voxels per step")
            extra["batched_3d_c5_large_step"] = strip(r)
        # the single 2-D pair: throughput, then its gradient descent and the
        # throughput at the momentum the descent reached
        w2 = {rho: synthetic.workload("c2", p0_kind="zero", rho=rho) for rho in (1.0, 0.5, 0.1)}
        w2r = synthetic.workload("c2", p0_kind="realistic")
        r = measure(w2r, "c2", max(args.steps, 20), args.warmup, 1, args.flags, autotune, torch, api)
        r["workload"] = "c2: " + WORKLOADS["c2"]
        extra["single_pair_c2"] = strip(r)
        extra["c2_descent"] = descent_c2(w2, args.descent_iters, max(args.steps, 20), torch, api)
        extra["forward_deformation"] = forward_deformation(wl, args.steps, args.warmup, torch, api)
        extra["lbfgs"] = lbfgs_rate(wl, 4, torch, api)
        extra["schemes"] = scheme_comparison(wl, args.steps, args.warmup, torch, api, synthetic)
        # the library's streaming copy at 1 GiB: the achievable-bandwidth reference
        extra["stream_copy_1GiB_GBps"] = copy_rate(1 << 30, torch, api)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_eval"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "pairs": len(wl.pairs),
                   "voxels": voxels, "T": wl.T, "p0": "realistic (smooth, a few tenths of a voxel per step)",
                   "flags": args.flags,
                   "mode": f"batched tile lists in {main_run['lanes']} concurrent lanes (one stream and one captured "
                           "HIP graph each), sqrt(T) checkpoints",
                   "tuning": tuning},
        "pair_evals_per_s": main_run["pair_evals_per_s"],
        "ms_per_step_median": main_run["ms_per_eval_median"],
        "ms_per_step_min": main_run["ms_per_eval_min"],
        "step_algorithmic_GBps": main_run["step_algorithmic_GBps"],
        "step_hbm_frac": main_run["step_hbm_frac"],
        "step_displacement_px": main_run["step_displacement_px"],
        "roofline": main_run["roofline"],
        "unfused": main_run.get("unfused"),
        "cpu_baseline": cpu,
        "extra": extra,
        "kernels": main_run["kernels"],
        "kernel_source_sha": kernel_source_sha(),
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
