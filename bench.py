#!/usr/bin/env python3
"""Benchmark of the EDAC-SPH wind-tunnel hot path on one MI355X.

A step is one explicit-midpoint RK2 step of the whole path (bin + Morton
sort, neighbour table, density, boundary values, force pass, stage updates,
time-average/transfer/re-spawn bookkeeping, drag) on the 2D channel workload
(4 x 1, dx = 0.01, 40,000 fluid particles, 5-layer inlet and hybrid outlet,
Gaussian pressure pulse of amplitude 0.01 rho0 c0 U at x = 2, width 0.1).

Metric: pair-interactions/s = (fluid-neighbour pairs per right-hand side) x 2
right-hand sides per step x steps / time, with the state resident in HBM.
Prints one JSON line. The roofline object reports the force kernel (the
dominant kernel) timed alone with HIP events on the library's stream; the
cpu_baseline object times the FP64 CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "pair-interactions/s of EDAC RHS (FP64 vs FP32 vs adjoint) + HBM roofline %"
WORKLOADS = {
    "C2": "2D channel 4x1 dx=0.01, 40k fluid + 5-layer inlet + 5-layer hybrid outlet, "
          "Gaussian pulse A=0.01 rho0 c0 U at x=2 w=0.1, Wendland C2 h=dx",
    "C1": "2D periodic box 1x1, 40x40 Taylor-Green, Wendland C2 h=dx",
    "C3": "2D cylinder D=2 Re=200 in 60x32, dx=D/50, 3-layer slip walls",
    "C4": "2D channel 4x1 dx=0.01 with D=0.2 cylinder, Re=20",
    "C5": "3D duct 4x1x1 dx=0.01, no-slip walls, inlet noise 1%",
    "C2Q": "2D channel 4x1 dx=0.01 with the C2 pulse, the paper's quintic spline "
           "(support 3h) at h=1.2 dx",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def force_bytes(sim, counts, types, prec_bytes):
    """Algorithmic HBM bytes of one force-pass launch: every array the kernel
    needs read once and every output written once (neighbour gathers that hit
    cache are not counted)."""
    import numpy as np
    D = sim.dim
    n = len(types)
    fb = (types == 0) | (types == 5)
    nfb = int(fb.sum())
    nnz = int(counts[fb].sum())
    pos = 8 * D if prec_bytes == 8 else 4 * D + 4  # FP32: cell offsets + packed cell
    rd = n * 1 + nfb * (pos + 2 * prec_bytes * D + 3 * prec_bytes + 4) + 4 * nnz
    wr = n * (2 * prec_bytes * D + 2 * prec_bytes) + int((types == 5).sum()) * 8 * D
    return rd + wr, dict(read=rd, write=wr, n=n, n_fluid_or_body=nfb, nnz=nnz)


def source_hash():
    h = hashlib.sha256()
    for f in ("pairs.hip", "sph_dev.h"):
        with open(os.path.join(ROOT, "paper_1907_04034_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload, prec):
    """HBM bytes per force launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"k_force_{workload}_{prec}_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    h = re.search(r"source_sha:\s*([0-9a-f]+)", txt)
    if not m or not h or h.group(1) != source_hash():
        return None
    return float(m.group(1))


def cpu_baseline(prm, s, budget_s):
    """The FP64 oracle as it stands, on the host's cores, over the first steps
    of the same workload until about budget_s seconds of stepping."""
    import numpy as np
    from oracle import oracle as O
    O.build(force=False)
    o = O.Oracle(prm, s)
    chunk = max(1, min(10, 400_000 // len(s["p"])))
    steps, pairs, elapsed = 0, 0, 0.0
    while elapsed < budget_s and steps < prm.get("steps", 2000):
        row, _ = o.neighbors()
        fl = o.state()["type"] == 0
        p_rhs = int((np.diff(row)[fl] - 1).sum())
        t1 = time.perf_counter()
        o.step(chunk)
        elapsed += time.perf_counter() - t1
        steps += chunk
        pairs += 2 * chunk * p_rhs
    return dict(value=pairs / elapsed, unit="pair-interactions/s", cores=O.num_threads(),
                kind="oracle",
                sample=f"FP64 oracle, first {steps} RK2 steps ({2 * steps} RHS) of the same "
                       f"workload, {elapsed:.1f} s of stepping")


def adjoint_bytes(sim, counts, types, prec_bytes):
    """Algorithmic HBM bytes of one reverse right-hand side (sph_rhs_adjoint):
    the forward state and stored derived fields read once per row, the weights
    and seeds read once, the neighbour indices read once per pass that walks
    them (pairs, neighbour average, boundary, density), every adjoint output
    written once. Re-reads of neighbour rows are served by cache and do not
    count."""
    D = sim.dim
    n = len(types)
    nnz = int(counts.sum())
    state = 8 * D + prec_bytes * (2 * D + 1) + 1 + 3 * prec_bytes  # x, u, ut, p, type, rho, V, pbar
    weights = prec_bytes * (2 * D + 1) + 8 * (1 + D + 3)  # abar, bbar, pdbar, seeds
    bnd = 8 * (D + 1) + 8 * 4 + 8  # averages, jcur/jprev, Shepard sum
    outputs = 8 * (3 * D + 1 + D + (D + 1) + 3)  # xbar, ubar, utbar, pbar, uinbar, avgbar, jprevbar
    internal = 2 * 8 * 10  # scratch written and read back between the four passes
    rd = n * (state + weights + bnd + internal // 2) + 4 * nnz * 4 + 4 * n * 4
    wr = n * (outputs + internal // 2)
    return rd + wr


def timed_launches(stream, reps, launch):
    """Average GPU time in ms of one call of `launch` over `reps` calls queued
    back to back on `stream` between one pair of HIP events (one pair per call
    would add the events' own cost, about 2.5 us, to every call)."""
    import torch
    launch()  # warm
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        launch()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def adjoint_bench(args):
    """Reverse of a run of steps on the channel-with-cylinder workload: the
    time-averaged-drag gradient (checkpointed forward, segment replay, reverse
    of every step). value = 2 P_RHS x steps / time of the reverse sweep (replay
    included)."""
    import numpy as np
    import torch
    from paper_1907_04034_amd import adjoint as A
    from paper_1907_04034_amd import binding as B
    from paper_1907_04034_amd import inputs as I

    torch.cuda.set_device(0)
    prm, s = I.config(args.config)
    K = args.steps
    log(f"bench adjoint: {prm['name']} n={len(s['p'])} prec={args.precision} steps={K}")
    stream = torch.cuda.current_stream()
    fbar = np.zeros((K, 3))
    fbar[:, 0] = 1.0 / K
    # warm-up: a short forward + reverse on its own simulation
    wsim = B.Simulation(prm, s, prec=args.precision)
    w = A.DragAdjoint(wsim, max(2, min(args.warmup, 20)), segment=args.segment)
    w.forward()
    w.backward(np.zeros((w.nsteps, 3)))
    if wsim.poll_error():
        raise SystemExit("device error during warm-up")
    del w, wsim
    sim = B.Simulation(prm, s, prec=args.precision)
    run = A.DragAdjoint(sim, K, segment=args.segment)
    torch.cuda.synchronize()
    times = {}
    for phase in ("forward", "backward"):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        w0 = time.perf_counter()
        e0.record(stream)
        if phase == "forward":
            hist = run.forward()
        else:
            run.backward(fbar)
        e1.record(stream)
        torch.cuda.synchronize()
        times[phase] = max(e0.elapsed_time(e1), 1e3 * (time.perf_counter() - w0))
        log(f"bench adjoint: {phase} {times[phase]:.1f} ms")
    if sim.poll_error():
        raise SystemExit("device error in the timed region")
    J = float(hist[:, 0].mean().item())
    # pairs per right-hand side at the start state (the reverse ends there)
    sim2 = B.Simulation(prm, s, prec=args.precision)
    sim2.bin()
    sim2.neighbors()
    sim2.rhs()
    cnt, _ = sim2.neighbor_table()
    types = sim2.state()["type"]
    p_rhs = int((cnt[types == 0] - 1).sum())
    value = 2 * p_rhs * K / (times["backward"] * 1e-3)
    # one reverse right-hand side, timed alone
    n = len(types)
    rng = np.random.default_rng(0)
    ab = rng.standard_normal((n, 3))
    sim2.rhs_adjoint(abar=ab, bbar=ab, pdbar=ab[:, 0], fbar=(1.0, 0.0, 0.0))
    torch.cuda.synchronize()
    reps = args.force_reps
    st_adj = sim2._adj_struct()
    a_us = 1e3 * timed_launches(stream, reps, lambda: sim2.rhs_adjoint_launch(st_adj))
    prec_bytes = 8 if args.precision == "fp64" else 4
    abytes = adjoint_bytes(sim2, cnt, types, prec_bytes)
    achieved = abytes / (a_us * 1e-6) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": min(args.warmup, 20),
        "ms_per_step": times["backward"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 pairs / f64 positions",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config] + ", gradient of the time-averaged drag "
                   "w.r.t. the inlet profile", "config": args.config, "form": "adjoint",
                   "particles": int(len(s["p"])), "pairs_per_rhs": p_rhs, "rhs_per_step": 2,
                   "precision": args.precision, "segment": run.segment,
                   "forward_ms": times["forward"], "backward_ms": times["backward"],
                   "J": J},
        "roofline": {"bound": "hbm", "kernel": "sph_rhs_adjoint (4 kernels)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": abytes, "launch_us": a_us},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--config", default="C2", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--force-reps", type=int, default=100)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run a plain device copy of this size (for counter scaling)")
    ap.add_argument("--form", default="forward", choices=["forward", "adjoint"],
                    help="adjoint: gradient of the time-averaged drag (default config C4)")
    ap.add_argument("--segment", type=int, default=50, help="adjoint checkpoint interval")
    ap.add_argument("--outlet", default="hybrid",
                    choices=["hybrid", "moc", "do-nothing", "mod-do-nothing", "mirror"],
                    help="outlet rule (forward form only)")
    ap.add_argument("--mirror-inlet", action="store_true",
                    help="inlet pressure mirrored from the fluid (forward form only)")
    ap.add_argument("--sort-every-step", action="store_true",
                    help="sort by cell at every step instead of keeping the cell order "
                         "while the skin allows")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this path runs on one GPU; --gpus must be 1"}))
        log("bench.py: the benchmark runs on one GPU; --gpus above 1 is not supported")
        sys.exit(2)
    if args.form == "adjoint":
        if args.outlet != "hybrid" or args.mirror_inlet:
            raise SystemExit("the adjoint form covers the hybrid outlet and the "
                             "characteristic inlet only")
        if args.config == "C2" and "--config" not in sys.argv:
            args.config = "C4"
        if "--steps" not in sys.argv:
            args.steps = 500
        adjoint_bench(args)
        return

    import numpy as np
    import torch
    from paper_1907_04034_amd import binding as B
    from paper_1907_04034_amd import inputs as I

    torch.cuda.set_device(0)
    prm, s = I.config(args.config)
    prm["outlet"] = I.OUTLETS[args.outlet]
    if args.mirror_inlet:
        prm["flags"] |= I.FLAG_MIRROR_INLET
    if not args.sort_every_step:
        prm["flags"] |= I.FLAG_REUSE_BINS
    log(f"bench: {prm['name']} n={len(s['p'])} prec={args.precision} "
        f"reuse_bins={not args.sort_every_step} outlet={args.outlet}")
    sim = B.Simulation(prm, s, prec=args.precision)
    stream = torch.cuda.current_stream()

    if args.copy_calibration_mib:
        nb = args.copy_calibration_mib << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"bench: copy calibration {nb} bytes x3 done")

    sim.step(args.warmup)
    bits = sim.poll_error()
    if bits:
        raise SystemExit(f"device error bits after warmup: {bits}")
    torch.cuda.synchronize()

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    gpu_ms = e0.elapsed_time(e1)
    bits = sim.poll_error()
    if bits:
        raise SystemExit(f"device error bits in timed region: {bits}")
    log(f"bench: {args.steps} steps in {gpu_ms:.2f} ms (events), {wall * 1e3:.2f} ms wall")

    # pairs per right-hand side, from the neighbour table of the last stage
    cnt, _ = sim.neighbor_table()
    st = sim.state()
    types = st["type"]
    fl = types == 0
    p_rhs = int((cnt[fl] - 1).sum())
    t_step = max(gpu_ms, wall * 1e3) / args.steps
    value = 2 * p_rhs / (t_step * 1e-3)

    # dominant kernel alone: fresh bin/neighbours/rhs, then force launches
    sim.bin()
    sim.neighbors()
    sim.rhs()
    cnt, _ = sim.neighbor_table()
    types = sim.state()["type"]
    torch.cuda.synchronize()
    reps = args.force_reps
    f_us = 1e3 * timed_launches(stream, reps, lambda: sim.force(reduce_drag=False))
    prec_bytes = 8 if args.precision == "fp64" else 4
    fbytes, fdetail = force_bytes(sim, cnt, types, prec_bytes)
    achieved = fbytes / (f_us * 1e-6) / 1e9
    traffic = traffic_from_profile(args.config, args.precision)
    log(f"bench: k_force {f_us:.2f} us/launch, {fbytes / 1e6:.2f} MB algorithmic, "
        f"{achieved:.1f} GB/s")

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 pairs / f64 positions",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "config": args.config,
                   "particles": int(len(s["p"])), "pairs_per_rhs": p_rhs,
                   "rhs_per_step": 2, "precision": args.precision, "outlet": args.outlet,
                   "inlet": "mirror" if args.mirror_inlet else "characteristic",
                   "cell_order": "sorted every step" if args.sort_every_step
                   else "kept while the cell skin allows"},
        "roofline": {"bound": "hbm", "kernel": "k_force", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "algorithmic_bytes_per_launch": fbytes,
                     "launch_us": f_us, "source_sha": source_hash()},
    }
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(prm, s, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
