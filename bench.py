#!/usr/bin/env python3
"""Throughput of the fused double-MRT step (flow + thermal + enthalpy) on one
MI355X, on the convection-melting cavity workload: 1024x1024 lattice, hot
left wall, cold right wall, adiabatic top/bottom, Ra = 1e6, Da = 1e-4,
Pr = 1, Ste = 1, porosity 0.4 with a seeded log-normal permeability
(sigma 0.1), initially solid (Sec. 4.3 setting at a new size).

Prints one JSON line: MLUPS over the timed steps, the roofline of the step
kernel (HIP events on the solver's stream), and the FP64 oracle timed on a
bounded sample on the host cores.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12  # MI355X HBM3E, bytes/s
# Algorithmic bytes per cell and launch (float32): a cell where the flow is
# solved reads and writes its 9 + 5 populations and f_l and reads the three
# porous fields; a solid cell moves only the 5 thermal populations, f_l and
# porosity.  A launch of one step moves them once per step; a launch of two
# steps reads the state k once and writes the state k+2 once (the state k+1
# stays on chip), so it moves them once per two steps.
BYTES_FLUID = 2 * (9 + 5) * 4 + 2 * 4 + 3 * 4   # 132
BYTES_SOLID = 2 * 5 * 4 + 2 * 4 + 4             # 52
# batched cavities have uniform porous fields: no per-node porous reads
BYTES_FLUID_BATCH = 2 * (9 + 5) * 4 + 2 * 4      # 120
BYTES_SOLID_BATCH = 2 * 5 * 4 + 2 * 4            # 48
KERNEL_SRC = [os.path.join(ROOT, "paper_1503_08406_amd", "csrc", n)
              for n in ("dmrt_step.hip", "dmrt_step2.hip", "dmrt_tile2.h", "dmrt_node.h",
                        "dmrt_device.h", "dmrt_internal.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_traffic_cavity1024.json")
TRAFFIC_FILE_4096 = os.path.join(ROOT, "profiles", "step_traffic_cavity4096.json")


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SRC:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def cpu_baseline(case, budget_s=15.0):
    """The FP64 oracle as it stands, on a bounded sample of the same workload
    (from its initial state: the oracle takes minutes to reach the GPU's
    timed window), on the host threads this process may use (at most 16, the
    CPU share of a one-GPU machine) and on one thread."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from conftest import oracle_from_case
    cores = min(16, len(os.sched_getaffinity(0)))
    o = oracle_from_case(case, nthreads=cores)
    t = time.perf_counter()
    o.step(5)
    dt = (time.perf_counter() - t) / 5
    n = max(5, min(2000, int(budget_s / max(dt, 1e-6))))
    t = time.perf_counter()
    o.step(n)
    el = time.perf_counter() - t
    cells = case["nx"] * case["ny"]
    o1 = oracle_from_case(case, nthreads=1)  # one thread, a short sample
    t = time.perf_counter()
    o1.step(3)
    el1 = time.perf_counter() - t
    return {"value": round(cells * n / el / 1e6, 3), "unit": "MLUPS", "cores": cores,
            "host_cores_available": len(os.sched_getaffinity(0)),
            "host_cpu_count": os.cpu_count(),
            "value_1_thread": round(cells * 3 / el1 / 1e6, 3),
            "kind": "oracle",
            "sample": "steps 5..%d of the %dx%d cavity from its initial state (FP64 oracle, "
                      "%d OpenMP threads, %.1f s)" % (5 + n, case["nx"], case["ny"], cores, el)}


def active_cell_steps(case, steps, samples, **over):
    """Untimed replay: integral over the timed steps of the number of cells
    where the flow is solved (trapezoid over `samples` points)."""
    from paper_1503_08406_amd.dmrt import Solver
    s = Solver(case, **over)
    pts = [(0, s.diag()["active"])]
    for k in range(1, samples + 1):
        tgt = steps * k // samples
        s.step(tgt - s.time)
        pts.append((tgt, s.diag()["active"]))
    tot = 0.0
    for (t0, a0), (t1, a1) in zip(pts, pts[1:]):
        tot += 0.5 * (a0 + a1) * (t1 - t0)
    s.close()
    return tot, pts[-1][1]


def small_configs():
    """The two small validation workloads in full, on the GPU (graph replay
    of 64 steps) and on the FP64 oracle (up to 16 threads): the conduction
    slab of Sec. 4.1 (256x4, 5000 steps) and the corner of Sec. 4.2 (256x256,
    20000 steps).  Wall-clock seconds of each; context for the oracle figure,
    not a throughput claim (both are far too small to fill the GPU)."""
    import torch
    from paper_1503_08406_amd import workloads as W
    from paper_1503_08406_amd.dmrt import Solver
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from conftest import oracle_from_case
    cores = min(16, len(os.sched_getaffinity(0)))
    out = {}
    for name, case in (("conduction_slab_256x4", W.conduction_slab()),
                       ("corner_256x256", W.corner())):
        steps = case["steps"]
        s = Solver(case, graph_steps=64)
        s.sync()
        torch.cuda.synchronize()
        t = time.perf_counter()
        s.step(steps)
        s.sync()
        g = time.perf_counter() - t
        s.close()
        o = oracle_from_case(case, nthreads=cores)
        t = time.perf_counter()
        o.step(steps)
        c = time.perf_counter() - t
        cells = case["nx"] * case["ny"]
        out[name] = {"steps": steps, "gpu_s": round(g, 4), "oracle_s": round(c, 3),
                     "oracle_cores": cores, "gpu_mlups": round(cells * steps / g / 1e6, 1),
                     "oracle_mlups": round(cells * steps / c / 1e6, 2)}
    return out


def lead_steps(gsteps, spl):
    """Untimed steps run right before a timed window (from a checkpoint taken
    that many steps earlier): one graph's worth, or two when a graph holds an
    odd number of launches, so that the window replays graphs captured for
    both buffer parities and starts on a device that is already busy (a few
    launches' worth without graphs)."""
    if not gsteps:
        return 4 * spl
    return gsteps * (2 if (gsteps // spl) % 2 else 1)


def window_accounting(case, buf, steps, samples, lead=0, **over):
    """Untimed replay of a timed window from the checkpoint `buf`, `lead`
    steps before the window: the integral over the window of the number of
    cells where the flow is solved (trapezoid over at most `samples` points)
    and the count at its end."""
    from paper_1503_08406_amd.dmrt import Solver
    s = Solver(case, **over)
    s.load(buf)
    s.step(lead)
    t0 = s.time
    samples = max(1, min(samples, steps))
    pts = [(0, s.diag()["active"])]
    for k in range(1, samples + 1):
        tgt = steps * k // samples
        s.step(t0 + tgt - s.time)
        pts.append((tgt, s.diag()["active"]))
    s.close()
    tot = sum(0.5 * (a0 + a1) * (t1 - t0_) for (t0_, a0), (t1, a1) in zip(pts, pts[1:]))
    return tot, pts[-1][1]


def repeats(case, buf, steps, lead, n=5, **over):
    """The timed window (`steps` steps, `lead` steps after the checkpoint
    `buf`) timed n more times, each on a fresh solver loaded from the
    checkpoint (HIP events on its stream): kernel times per step and their
    median.  Each solver runs the `lead` steps untimed right before the
    window, as the main run does, so that graph capture stays out of the
    timed region."""
    import torch
    from paper_1503_08406_amd.dmrt import Solver
    ms = []
    for _ in range(n):
        s = Solver(case, **over)
        s.load(buf)
        s.step(lead)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(s.stream)
        s.step(steps)
        ev1.record(s.stream)
        s.sync()
        ms.append(ev0.elapsed_time(ev1) / steps)
        s.close()
    return {"n": n, "steps": steps, "kernel_ms": [round(v, 6) for v in ms],
            "median_kernel_ms": round(sorted(ms)[n // 2], 6)}


def step_kernel(spl):
    """Name of the step kernel that a solver advancing spl steps per launch
    runs (the default launch shape)."""
    return ("k_step2 (two steps per launch, tiles of 62 x 6 nodes)" if spl == 2
            else "k_step (flow, 4 rows, 1 node per lane)")


def plain_copy(nbytes, copies=64, reps=10):
    """What a plain device copy reaches for the same bytes: copies back and
    forth between two buffers of nbytes/2 each (each copy reads half and
    writes half), replayed from a graph and timed with HIP events.  This is
    the rate a pure stream of this traffic and working-set size attains on
    the device, next to the nominal HBM peak."""
    import torch
    n = max(1, int(nbytes) // 8)  # floats per buffer
    a = torch.ones(n, device="cuda")
    b = torch.zeros(n, device="cuda")
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for _ in range(4):
            b.copy_(a)
            a.copy_(b)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            for _ in range(copies // 2):
                b.copy_(a)
                a.copy_(b)
        g.replay()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            g.replay()
        e1.record(st)
    e1.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / (reps * copies)
    del g, a, b
    return {"bytes": 8 * n, "us": round(us, 3), "GBps": round(8 * n / (us * 1e-6) / 1e9, 1)}


def hbm_point(n=4096, steps=1000, warmup=100, graph_steps=64, steps_per_launch=2):
    """The cavity workload at n x n (4096^2: 2.5 GB of state, past the
    Infinity Cache, so the step streams from HBM), timed like the main run;
    roofline with the same phase-mixed byte model, per launch."""
    import torch
    from paper_1503_08406_amd import workloads as W
    from paper_1503_08406_amd.dmrt import Solver
    case = W.cavity(nx=n, ny=n, steps=steps)
    s = Solver(case, graph_steps=graph_steps, steps_per_launch=steps_per_launch)
    spl = s.launch_steps
    s.step(warmup)
    s.sync()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(s.stream)
    s.step(steps)
    ev1.record(s.stream)
    s.sync()
    wall = time.perf_counter() - t0
    kern_ms = ev0.elapsed_time(ev1) / steps
    d = s.diag()
    s.close()
    act_steps, _ = active_cell_steps(case, warmup + steps, 20, graph_steps=graph_steps)
    cells = n * n
    ff = act_steps / (cells * (warmup + steps))
    bpl = (BYTES_FLUID * ff + BYTES_SOLID * (1 - ff)) * cells
    launch_ms = kern_ms * spl
    cp = plain_copy(bpl)
    cp["frac_of_copy"] = round(cp["us"] / (launch_ms * 1e3), 3)
    # measured HBM traffic of this kernel at this size (rocprofv3 FETCH_SIZE /
    # WRITE_SIZE over steps 10..210), valid while the kernel source is the one
    # that was measured; its liquid fraction is stated beside it
    traffic = None
    if n == 4096 and os.path.exists(TRAFFIC_FILE_4096):
        tr = json.load(open(TRAFFIC_FILE_4096))
        if tr.get("kernel_sha") == kernel_hash():
            traffic = {"bytes": tr["bytes_per_launch"], "fluid_fraction": tr["fluid_fraction"],
                       "GBps": round(tr["bytes_per_launch"] / (launch_ms * 1e-3) / 1e9, 1)}
    return {"workload": "the same cavity at %dx%d (%.2f GB of state), steps %d..%d"
                        % (n, n, cells * 156 / 1e9, warmup, warmup + steps),
            "value": round(cells * steps / wall / 1e6, 2), "unit": "MLUPS",
            "kernel_ms_per_step": round(kern_ms, 6), "steps_per_launch": spl,
            "roofline": {"bound": "hbm", "achieved": round(bpl / (launch_ms * 1e-3) / 1e9, 1),
                         "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                         "frac": round(bpl / (launch_ms * 1e-3) / HBM_PEAK, 4),
                         "kernel": step_kernel(spl), "kernel_ms": round(launch_ms, 6),
                         "bytes_per_launch": round(bpl),
                         "fluid_fraction_mean": round(ff, 5), "traffic": traffic,
                         "plain_copy": cp},
            "nonfinite": int(d["nonfinite"])}


def flow_point(n=4096, steps=256, warmup=64, graph_steps=64, steps_per_launch=2):
    """The cavity workload at n x n started liquid (initial theta 0.5, above
    the liquidus), so that the flow part of the step (D2Q9 pulls, closure,
    collision) runs at nearly every node, on a state far beyond the Infinity
    Cache: the HBM roofline of the fluid byte model (132 B per node and
    launch)."""
    import torch
    from paper_1503_08406_amd import workloads as W
    from paper_1503_08406_amd.dmrt import Solver
    case = W.cavity(nx=n, ny=n, steps=steps, T_init=0.5)
    over = dict(graph_steps=graph_steps, steps_per_launch=steps_per_launch)
    s = Solver(case, **over)
    spl = s.launch_steps
    lead = min(lead_steps(graph_steps, spl), warmup)
    s.step(warmup - lead)
    s.sync()
    buf = s.save()  # lead steps before the window
    s.step(lead)
    s.sync()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(s.stream)
    s.step(steps)
    ev1.record(s.stream)
    s.sync()
    wall = time.perf_counter() - t0
    kern_ms = ev0.elapsed_time(ev1) / steps
    d = s.diag()
    s.close()
    act, act_end = window_accounting(case, buf, steps, 16, lead, **over)
    rep = repeats(case, buf, steps, lead, n=3, **over)
    one = repeats(case, buf, steps, lead, n=3, graph_steps=graph_steps, steps_per_launch=1)
    del buf
    cells = n * n
    ff = act / (cells * steps)
    bpl = (BYTES_FLUID * ff + BYTES_SOLID * (1 - ff)) * cells
    launch_ms = rep["median_kernel_ms"] * spl
    one_ms = one["median_kernel_ms"]
    return {"workload": "the same cavity at %dx%d started liquid (initial theta 0.5), steps "
                        "%d..%d" % (n, n, warmup, warmup + steps),
            "value": round(cells * steps / wall / 1e6, 2), "unit": "MLUPS",
            "kernel_ms_per_step": round(kern_ms, 6), "steps_per_launch": spl,
            "roofline": {"bound": "hbm", "achieved": round(bpl / (launch_ms * 1e-3) / 1e9, 1),
                         "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                         "frac": round(bpl / (launch_ms * 1e-3) / HBM_PEAK, 4),
                         "kernel": step_kernel(spl), "kernel_ms": round(launch_ms, 6),
                         "bytes_per_launch": round(bpl), "fluid_fraction_mean": round(ff, 5),
                         "bytes_per_cell": {"fluid": BYTES_FLUID, "solid": BYTES_SOLID},
                         "repeats": rep},
            "one_step_per_launch": {"kernel": step_kernel(1), "kernel_ms": round(one_ms, 6),
                                    "frac": round(bpl / (one_ms * 1e-3) / HBM_PEAK, 4),
                                    "repeats": one},
            "nonfinite": int(d["nonfinite"])}


def batched(single_mlups, steps=None, trial_steps=128, samples=20, store_hint=0, graph_steps=64):
    """The batched workload: 512 cavities of seeded uneven sizes and
    parameters (seed 4), advanced together for 10000 steps with the tuned
    launch shape (one step per launch, or two: rows 0) and graph replay of
    64 steps; the phase mix for the byte count comes from an untimed
    replay."""
    import torch
    from paper_1503_08406_amd import workloads as W
    from paper_1503_08406_amd.dmrt import BatchSolver
    cavs, opts, nsteps = W.cavity_batch()
    steps = steps or nsteps
    b = BatchSolver(cavs, graph_steps=graph_steps, store_hint=store_hint, **opts)
    rows, blocks, tune_ms = b.tune(trial_steps=trial_steps)
    spl = 2 if rows == 0 else 1
    cells = b.cells
    b.sync()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(b.stream)
    b.step(steps)
    ev1.record(b.stream)
    b.sync()
    wall = time.perf_counter() - t0
    kern_ms = ev0.elapsed_time(ev1) / steps
    liq, bad = b.check()
    assert (bad == 0).all(), "non-finite state in the batch"
    b.close()
    # phase accounting replay
    r = BatchSolver(cavs, graph_steps=graph_steps, store_hint=store_hint, **opts)
    r.set_launch(rows, blocks)
    pts = [(0, int(r.check()[0].sum()))]
    for k in range(1, samples + 1):
        tgt = steps * k // samples
        r.step(tgt - r.time)
        pts.append((tgt, int(r.check()[0].sum())))
    r.close()
    act = sum(0.5 * (a0 + a1) * (t1 - t0_) for (t0_, a0), (t1, a1) in zip(pts, pts[1:]))
    ff = act / (cells * steps)
    bpl = (BYTES_FLUID_BATCH * ff + BYTES_SOLID_BATCH * (1 - ff)) * cells
    launch_ms = kern_ms * spl
    mlups = cells * steps / wall / 1e6
    return {"workload": "512 convection-melting cavities (Sec. 4.3 setting), nx, ny iid in "
                        "[64, 512], Ra 10^U(4,6), Da 10^U(-5,-2), eps U(0.3,0.9), Ste U(0.1,2), "
                        "Pr 1, seed 4, uniform porous fields per cavity, steps 0..%d" % steps,
            "cavities": len(cavs), "cells": int(cells), "steps": steps,
            "value": round(mlups, 2), "unit": "MLUPS",
            "ms_per_step": round(wall * 1e3 / steps, 6),
            "ratio_to_single": round(mlups / single_mlups, 4),
            "launch": {"rows": rows, "blocks": blocks, "graph_steps": graph_steps,
                       "steps_per_launch": spl,
                       "tuner_trial_ms_per_step": round(tune_ms, 6)},
            "roofline": {"bound": "hbm", "achieved": round(bpl / (launch_ms * 1e-3) / 1e9, 1),
                         "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                         "frac": round(bpl / (launch_ms * 1e-3) / HBM_PEAK, 4),
                         "kernel": "k_batch_step2" if spl == 2 else "k_batch_step",
                         "kernel_ms": round(launch_ms, 6), "kernel_ms_per_step": round(kern_ms, 6),
                         "bytes_per_launch": round(bpl), "fluid_fraction_mean": round(ff, 5),
                         "bytes_per_cell": {"fluid": BYTES_FLUID_BATCH, "solid": BYTES_SOLID_BATCH}},
            "liquid_cells_end": int(liq.sum())}


def adjoint_timing(warm=200, steps=0, record_mode=0):
    """The inverse-problem workload (512x512 cavity, Gaussian-random-field
    log K seed 1, target run seed 2, 2000 steps): wall time of the plain
    forward run, of the recorded forward run and of the adjoint (the
    reversed steps, plus the segment recomputation when only checkpoints are
    kept), all from the initial state.  record_mode 0 keeps every state of the
    run when it fits (here 38 GB of HBM), 1 keeps checkpoints every
    ceil(sqrt n) steps.  The first record and adjoint calls capture their HIP
    graphs; the second, timed ones replay them (as an optimisation loop
    does)."""
    import numpy as np
    from paper_1503_08406_amd import workloads as W
    from paper_1503_08406_amd.dmrt import Solver
    case, target = W.adjoint_cavity(), W.adjoint_cavity(seed=2)
    steps = steps or case["steps"]
    t = Solver(target, graph_steps=64)
    t.step(steps)
    Ft = t.fields()
    t.close()
    s = Solver(case, graph_steps=64, record_mode=record_mode)
    s.step(warm)
    s.sync()

    def timed(fn):
        s.sync()
        t0 = time.perf_counter()
        fn()
        s.sync()
        return (time.perf_counter() - t0) * 1e3

    s.reset()
    fwd = timed(lambda: s.step(steps))
    # the same forward run at one step per launch (context: the run before
    # two-step launches, and what the adjoint's cost was first quoted against)
    s1 = Solver(case, graph_steps=64, steps_per_launch=1)
    s1.step(warm)
    s1.reset()
    s1.sync()
    t0 = time.perf_counter()
    s1.step(steps)
    s1.sync()
    fwd1 = (time.perf_counter() - t0) * 1e3
    s1.close()
    s.reset()
    rec_first = timed(lambda: s.record(steps))  # captures the recording's graph
    s.reset()
    rec = timed(lambda: s.record(steps))
    F = s.fields()
    dT, dfl = F["T"] - Ft["T"], F["fl"] - Ft["fl"]
    loss = 0.5 * (float(np.sum(dT.astype(np.float64) ** 2)) + float(np.sum(dfl.astype(np.float64) ** 2)))
    out = {}
    adj_first = timed(lambda: out.setdefault("g0", s.adjoint(dT, dfl)))  # builds the graph
    adj = timed(lambda: out.setdefault("g", s.adjoint(dT, dfl)))
    gk, ge = out["g"]
    assert np.array_equal(gk, out["g0"][0]) and np.array_equal(ge, out["g0"][1])
    s.close()
    return {"workload": "inverse problem: 512x512 cavity (Sec. 4.3 setting), Ra=1e5 Da=1e-3 Ste=1 "
                        "eps=0.4, log K = log(Da H^2) + 0.5 GRF(corr 32, seed 1), target run "
                        "seed 2, L = 1/2 sum((f_l - f_l*)^2 + (T - T*)^2) after %d steps" % steps,
            "record_mode": {0: "every state kept (fits in HBM)", 1: "sqrt(n) checkpoints, "
                            "segments recomputed"}[record_mode],
            "steps": steps, "forward_ms": round(fwd, 3),
            "forward_one_step_per_launch_ms": round(fwd1, 3), "record_ms": round(rec, 3),
            "record_first_call_ms": round(rec_first, 3),
            "adjoint_ms": round(adj, 3), "adjoint_first_call_ms": round(adj_first, 3),
            "adjoint_over_forward": round(adj / fwd, 3),
            "record_and_adjoint_over_forward": round((rec + adj) / fwd, 3),
            "record_and_adjoint_over_forward_one_step_per_launch": round((rec + adj) / fwd1, 3),
            "loss": loss, "grad_logK_norm": float(np.linalg.norm(gk)),
            "grad_eps_norm": float(np.linalg.norm(ge)),
            "liquid_cells_end": int((F["fl"] > 0).sum())}


# Literal readings of the thermal model against the default ones, on the
# paper's own Sec. 4.3 problem (gallium in glass beads, 200 x 200).  The
# ratios are fitted to the values the paper quotes there: Eq. (7) with
# c_ps/c_pl and the matrix capacity that give sigma = 0.8604 (liquid) and
# 0.8352 (solid) at porosity 0.385, Eq. (8) with k_s = k_l and the matrix
# conductivity that gives lambda = k_e/k_l = 0.2719 in the liquid.
CPS_GA, CM_GA = 0.9345454545, 0.7730081301
KM_GA = 0.0299507727
ABLATION = [
    ("default", {}),
    ("sigma_eq7", dict(sigma_mode=1, cps_ratio=CPS_GA, cm_ratio=CM_GA)),
    ("ke_eq8", dict(ke_mode=1, ks_ratio=1.0, km_ratio=KM_GA)),
    ("r2", dict(latent_mode=1)),
    ("all_literal", dict(sigma_mode=1, cps_ratio=CPS_GA, cm_ratio=CM_GA, ke_mode=1, ks_ratio=1.0,
                         km_ratio=KM_GA, latent_mode=1)),
]


def ablation(horizons=((0.04, True), (0.457, True), (1.829, False)), graph_steps=64):
    """Run every reading to each Fourier number of `horizons` (the R2
    readings only where the flag says so) and print one JSON line per
    (reading, Fo): time per step, melted fraction, the front (mean, top and
    bottom rows), the range of T, and the largest differences of T and f_l
    from the default readings."""
    import numpy as np
    import torch
    from paper_1503_08406_amd import workloads as W
    from paper_1503_08406_amd.dmrt import Solver
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from conftest import front_rows

    from paper_1503_08406_amd.dmrt import derive
    torch.cuda.set_device(0)
    case = W.gallium_cavity()
    # time steps of a Fourier number t alpha_l / H^2, alpha_l from the
    # library's Sec. 4.3 mapping of (Ra, Pr, Ma, H)
    alpha_l = derive(case["nx"], case["ny"], case["Ra"], case["Da"], case["Pr"], case["Ste"],
                     H=case["H"], **case["opts"])["alpha_l"]
    ref = {}
    for fo, with_r2 in horizons:
        steps = int(round(fo * case["H"] ** 2 / alpha_l))
        for name, over in ABLATION:
            if over.get("latent_mode") and not with_r2:
                continue  # R2 sweeps the whole lattice many times a step
            s = Solver(case, graph_steps=graph_steps, **over)
            s.step(graph_steps)  # graph capture outside the timing
            s.sync()
            t = time.perf_counter()
            s.step(steps - graph_steps)
            s.sync()
            el = time.perf_counter() - t
            F = s.fields()
            d = s.diag()
            fr = front_rows(F["fl"])
            row = {"reading": name, "Fo": fo, "steps": steps,
                   "us_per_step": round(el * 1e6 / (steps - graph_steps), 2),
                   "melted": round(float(F["fl"].mean()), 5),
                   "front_mean": round(float(fr.mean()), 3),
                   "front_top": round(float(fr[-10:].mean()), 3),
                   "front_bottom": round(float(fr[:10].mean()), 3),
                   "T_min": round(float(F["T"].min()), 4), "T_max": round(float(F["T"].max()), 4),
                   "u_max": float("%.4g" % d["u_max"]), "nonfinite": int(d["nonfinite"])}
            if name == "default":
                ref[fo] = F
            else:
                R = ref[fo]
                row["dT_max"] = float("%.4g" % np.abs(F["T"] - R["T"]).max())
                row["dfl_max"] = float("%.4g" % np.abs(F["fl"] - R["fl"]).max())
                row["dfront_mean"] = round(float(np.abs(fr - front_rows(R["fl"])).mean()), 3)
            print(json.dumps(row), flush=True)
            s.close()
    return 0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed steps")
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed steps right before the timed window")
    ap.add_argument("--start", type=int, default=50000,
                    help="untimed steps from the initial state to the timed window (half of "
                         "the workload's 100000, so that the window sees the melted, "
                         "convecting cavity)")
    ap.add_argument("--n", type=int, default=1024, help="lattice side")
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="steps per HIP graph in the timed window (0: plain launches, "
                         "measured faster on the 1024^2 lattice)")
    ap.add_argument("--block-rows", type=int, default=0, help="step-kernel block rows (0: auto)")
    ap.add_argument("--cells-per-lane", type=int, default=0, help="nodes per lane (0: auto)")
    ap.add_argument("--steps-per-launch", type=int, default=2,
                    help="time steps per launch of the step kernel (1 or 2)")
    ap.add_argument("--T-init", type=float, default=0.0,
                    help="initial temperature (0: solid start as in the workload; "
                         "0.5: liquid start, the flow is solved almost everywhere)")
    ap.add_argument("--store-hint", type=int, default=0,
                    help="cache policy of the state stores: 0 by working set, 1 plain, "
                         "2 write-through, 3 streaming")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-cavity measurement")
    ap.add_argument("--batch-steps", type=int, default=0, help="batched steps (0: the workload's)")
    ap.add_argument("--batch-graph-steps", type=int, default=64,
                    help="graph replay length of the batch (0: plain launches, for counter runs)")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing")
    ap.add_argument("--adjoint-steps", type=int, default=0,
                    help="steps of the adjoint run (0: the workload's 2000; fewer for profiling)")
    ap.add_argument("--no-hbm", action="store_true",
                    help="skip the 4096^2 points (state beyond the Infinity Cache)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--ablation", action="store_true",
                    help="instead of the benchmark: the readings of the thermal model on "
                         "the paper's Sec. 4.3 problem, one JSON line each")
    ap.add_argument("--ablation-fo", type=float, default=0.0,
                    help="with --ablation: one horizon, this Fourier number, all readings")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU; --gpus %d is not supported (the "
              "multi-GPU sharding is designed, not implemented)" % args.gpus, file=sys.stderr)
        return 2
    if args.ablation:
        return ablation(((args.ablation_fo, True),)) if args.ablation_fo > 0 else ablation()

    import torch
    from paper_1503_08406_amd import workloads as W
    from paper_1503_08406_amd.dmrt import Solver

    torch.cuda.set_device(0)
    case = W.cavity(nx=args.n, ny=args.n, steps=args.start + args.warmup + args.steps,
                    T_init=args.T_init)
    # plain launches by default: the host keeps ahead of 18 us launches, and
    # a graph's kernels ran 4 % slower in 20-step windows, 0-1 % in 2000-step
    # ones.  With --graph-steps, graphs of at most the window's length (even).
    gsteps = min(args.graph_steps, args.steps // 2 * 2)
    over = dict(graph_steps=gsteps, block_rows=args.block_rows, store_hint=args.store_hint,
                cells_per_lane=args.cells_per_lane, steps_per_launch=args.steps_per_launch)

    if args.copy_probe:
        a = torch.ones(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print("copy probe: 3 x 1 GiB device-to-device copies", flush=True)
        del a, b

    # untimed: advance to the start of the window, then the warm-up steps.
    # The checkpoint for the replays below is taken `lead` steps before the
    # window; those last steps run right before it (in the replays as well),
    # so that the window replays graphs captured for both buffer parities and
    # starts on a busy device.
    s = Solver(case, **over)
    spl = s.launch_steps
    pre = args.start + args.warmup
    lead = min(lead_steps(gsteps, spl), pre)
    s.step(pre - lead)
    s.sync()
    buf = s.save()
    s.step(lead)
    t_start = pre
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(s.stream)  # after the warm-up steps, outside the wall-clock bracket
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    ev1.record(s.stream)
    torch.cuda.synchronize()  # the whole device, the solver's stream included
    t1 = time.perf_counter()
    wall = t1 - t0
    kern_ms = ev0.elapsed_time(ev1) / args.steps
    d = s.diag()
    s.close()
    assert d["nonfinite"] == 0, "non-finite state after the timed run"
    cells = case["nx"] * case["ny"]
    mlups = cells * args.steps / wall / 1e6

    act_steps, act_end = window_accounting(case, buf, args.steps, 50, lead, **over)
    fluid_frac = act_steps / (cells * args.steps)
    bytes_per_launch = (BYTES_FLUID * fluid_frac + BYTES_SOLID * (1 - fluid_frac)) * cells
    rep = repeats(case, buf, args.steps, lead, **over)
    one = None
    if spl == 2:
        one = repeats(case, buf, args.steps, lead, n=3, **dict(over, steps_per_launch=1))
    del buf
    med_ms = rep["median_kernel_ms"]  # per step
    launch_ms = med_ms * spl
    achieved = bytes_per_launch / (launch_ms * 1e-3)
    # measured HBM traffic per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE, two
    # phase mixes solved for bytes per solid and per liquid node), valid while
    # the step kernel source is the one that was measured
    traffic = None
    if os.path.exists(TRAFFIC_FILE) and args.n == 1024:
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("kernel_sha") == kernel_hash():
            traffic = round((tr["bytes_per_cell_solid"] * (1 - fluid_frac) +
                             tr["bytes_per_cell_fluid"] * fluid_frac) * cells)

    cp = plain_copy(traffic or bytes_per_launch)
    cp["frac_of_copy"] = round(cp["us"] / (launch_ms * 1e3), 3)

    out = {
        "metric": "MLUPS (flow+thermal)",
        "value": round(mlups, 2),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "convection melting in a porous cavity %dx%d (Sec. 4.3 setting): "
                               "Ra=1e6 Da=1e-4 Pr=1 Ste=1 eps=0.4, log-normal K (sigma 0.1, "
                               "seed 3), initial theta %g, timed steps %d..%d"
                               % (args.n, args.n, args.T_init, t_start, t_start + args.steps),
                   "nx": args.n, "ny": args.n, "window_start": t_start,
                   "graph_steps": gsteps, "block_rows": args.block_rows,
                   "cells_per_lane": args.cells_per_lane, "steps_per_launch": spl,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": round(achieved / 1e9, 1), "peak": HBM_PEAK / 1e9,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK, 4),
                     "traffic": traffic,
                     "traffic_GBps": None if traffic is None else round(traffic / (launch_ms * 1e-3) / 1e9, 1),
                     "kernel": step_kernel(spl), "steps_per_launch": spl,
                     "kernel_ms": round(launch_ms, 6), "kernel_ms_per_step": round(med_ms, 6),
                     "kernel_ms_per_step_timed_run": round(kern_ms, 6),
                     "bytes_per_launch": round(bytes_per_launch),
                     "fluid_fraction_mean": round(fluid_frac, 5),
                     "bytes_per_cell": {"fluid": BYTES_FLUID, "solid": BYTES_SOLID},
                     "plain_copy": cp, "repeats": rep},
        "phase": {"active_cells_end": int(act_end), "front_mean_end": round(d["front_mean"], 3)},
    }
    if one is not None:
        one_ms = one["median_kernel_ms"]
        out["roofline"]["one_step_per_launch"] = {
            "kernel": step_kernel(1), "kernel_ms": round(one_ms, 6),
            "frac": round(bytes_per_launch / (one_ms * 1e-3) / HBM_PEAK, 4), "repeats": one}
    if not args.no_hbm:
        out["hbm_point"] = hbm_point(steps_per_launch=args.steps_per_launch)
        out["flow_point"] = flow_point(steps_per_launch=args.steps_per_launch)
    if not args.no_batch:
        out["batched"] = batched(mlups, steps=args.batch_steps or None, store_hint=args.store_hint,
                                 graph_steps=args.batch_graph_steps)
        if "hbm_point" in out:
            out["batched"]["ratio_to_single_4096"] = round(
                out["batched"]["value"] / out["hbm_point"]["value"], 4)
    if not args.no_adjoint:
        out["adjoint"] = adjoint_timing(steps=args.adjoint_steps)
        out["adjoint_checkpointed"] = adjoint_timing(steps=args.adjoint_steps, record_mode=1)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case)
        out["cpu_baseline"]["small_configs"] = small_configs()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
