#!/usr/bin/env python3
"""Benchmark of the EDAC-SPH wind-tunnel hot path on one MI355X.

A step is one explicit-midpoint RK2 step of the whole path (bin + Morton
sort, neighbour table, density, boundary values, force pass, stage updates,
time-average/transfer/re-spawn bookkeeping) with the state resident in HBM.
The default workload is the largest single-GPU configuration: the 3D duct
4 x 1 x 1, dx = 0.01 (4.0M fluid particles, 5-layer inlet and hybrid outlet,
3-layer no-slip walls, 1 % seeded inlet noise; 4.6M particles in all).

Metric: pair-interactions/s = (fluid-neighbour pairs per right-hand side) x 2
right-hand sides per step x steps / time. The line's value is the FP64 path;
the FP32 path (FP32 pair arithmetic on cell-relative offsets, FP64
sums) and the adjoint (one reverse right-hand side) are reported beside it
under "forms". The roofline object reports the force pass, timed alone with
HIP events on the library's stream, against the algorithmic bytes per
particle of the hot-path scope table (156 B in 3D FP64: x, u, ut, p, V, rho,
type in, a, b, pdot out), with the implementation's own byte count beside it;
cpu_baseline times the FP64 CPU oracle on a bounded sample of the workload,
on one host thread and on all of them.
"""
from __future__ import annotations

import argparse
import ctypes
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3}
METRIC = "pair-interactions/s of EDAC RHS (FP64 vs FP32 vs adjoint) + HBM roofline %"
WORKLOADS = {
    "C5": "3D duct 4x1x1 dx=0.01 (4.0M fluid + 5-layer inlet + 5-layer hybrid outlet + "
          "3-layer no-slip walls = 4.6M particles), uniform inlet u=1 with seeded 1% noise, "
          "Wendland C2 h=dx",
    "C2": "2D channel 4x1 dx=0.01, 40k fluid + 5-layer inlet + 5-layer hybrid outlet, "
          "Gaussian pulse A=0.01 rho0 c0 U at x=2 w=0.1, Wendland C2 h=dx",
    "C1": "2D periodic box 1x1, 40x40 Taylor-Green, Wendland C2 h=dx",
    "C3": "2D cylinder D=2 Re=200 in 60x32, dx=D/50, 3-layer slip walls",
    "C4": "2D channel 4x1 dx=0.01 with D=0.2 cylinder, Re=20",
    "C2Q": "2D channel 4x1 dx=0.01 with the C2 pulse, the paper's quintic spline "
           "(support 3h) at h=1.2 dx",
}
# Algorithmic bytes per particle per right-hand side (every array the pass
# needs read once, every output written once; neighbour re-reads served by
# LDS or cache not counted): pass D = neighbours + density, pass F = force.
# FP32 3D splits its 112 B total the way the 2D rows split.
SCOPE_BYTES = {(2, "fp64"): (36, 116), (3, "fp64"): (44, 156),
               (2, "fp32"): (24, 64), (3, "fp32"): (28, 84)}
# Algorithmic flops per ordered neighbour pair of the force pass (neighbour
# average 6, pair terms 75, one square root and two divisions counted once).
FORCE_FLOPS_PER_PAIR = 84


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def force_bytes(counts, types, prec_bytes, dim):
    """The implementation's own byte count of one force launch: each fluid or
    body row's own fields (position or cell offsets, u, ut, p, rho, V), count
    and table entries; every row's neighbour data read once (its record, 96
    bytes in 3D FP64 and 48 in FP32, or in 2D FP64 its position, u, ut, p,
    Shepard sum and kind) and its kind byte; the writes of a, b, pdot and
    pbar and of the body force."""
    fb = (types == 0) | (types == 5)
    n = len(types)
    nfb = int(fb.sum())
    nnz = int(counts[fb].sum())
    pos = 8 * dim if prec_bytes == 8 else 4 * dim + 4  # FP32: cell offsets + packed cell
    own = pos + 2 * prec_bytes * dim + 3 * prec_bytes + 4
    if prec_bytes == 4 or dim == 3:
        nbr = 96 if prec_bytes == 8 else 48
    else:
        nbr = 8 * dim + 2 * prec_bytes * dim + 2 * prec_bytes + 1
    rd = n * (1 + nbr) + nfb * own + 4 * nnz
    wr = n * (2 * prec_bytes * dim + 2 * prec_bytes) + int((types == 5).sum()) * 8 * dim
    return rd + wr


def code_text(src):
    """C++/HIP source without its comments and whitespace (string and
    character literals kept as written): what the compiled kernels depend on."""
    out, i, n = [], 0, len(src)
    while i < n:
        c = src[i]
        if c in "\"'":
            j = i + 1
            while j < n and src[j] != c:
                j += 2 if src[j] == "\\" else 1
            out.append(src[i:j + 1])
            i = j + 1
        elif src.startswith("//", i):
            i = src.find("\n", i)
            i = n if i < 0 else i
        elif src.startswith("/*", i):
            i = src.find("*/", i + 2)
            i = n if i < 0 else i + 2
        else:
            if not c.isspace():
                out.append(c)
            i += 1
    return "".join(out)


def source_hash():
    """Hash of the kernel sources' code (comments and whitespace left out), so
    that a counter summary stays valid across edits of comments only."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1907_04034_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(csrc, f), encoding="utf-8") as fh:
                h.update(code_text(fh.read()).encode())
    return h.hexdigest()[:16]


def counters_summary(workload, prec):
    """Traffic and limiter of the force pass from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", f"k_force_{workload}_{prec}_counters.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    h = re.search(r"source_sha:\s*([0-9a-f]+)", txt)
    if not h or h.group(1) != source_hash():
        return None
    out = {}
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if m:
        out["traffic"] = float(m.group(1))
    m = re.search(r"limiter:\s*(hbm|alu)\b", txt)
    if m:
        out["bound"] = m.group(1)
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_sample(prm, s, xmax):
    """The workload's particles with x < xmax (inlet, walls and fluid of the
    first stretch of the tunnel): a bounded sample of the same structure."""
    import numpy as np
    keep = s["x"][:, 0] < xmax
    t = {k: np.ascontiguousarray(v[keep]) for k, v in s.items()}
    t["id"] = np.arange(int(keep.sum()), dtype=np.int64)
    return t


def cpu_baseline(prm, s, args):
    """The FP64 oracle as it stands: one right-hand side (neighbour lists,
    density, boundary values, force pass) on a sample of the workload, timed
    on one host thread and on all of them; pair-interactions/s."""
    import numpy as np
    from oracle import oracle as O
    O.build(force=False)
    if prm["dim"] == 3:
        t = oracle_sample(prm, s, args.cpu_sample_x)
        what = f"the first {args.cpu_sample_x:g} m of the duct ({len(t['p'])} particles)"
    else:
        t = s
        what = f"the whole workload ({len(t['p'])} particles)"
    o = O.Oracle(prm, t)
    row, _ = o.neighbors()
    fl = o.state()["type"] == 0
    p_rhs = int((np.diff(row)[fl] - 1).sum())
    out = {}
    allt = os.cpu_count() or 1
    for label, nt in (("all", allt), ("one", 1)):
        O.set_threads(nt)
        reps, elapsed = 0, 0.0
        budget = args.cpu_budget if label == "all" else 2 * args.cpu_budget
        while elapsed < budget / 2 and reps < 20:
            t1 = time.perf_counter()
            o.rhs()
            elapsed += time.perf_counter() - t1
            reps += 1
        out[label] = (p_rhs * reps / elapsed, nt, reps, elapsed)
    O.set_threads(allt)
    v_all, n_all, r_all, e_all = out["all"]
    v_one, _, r_one, e_one = out["one"]
    return dict(value=v_all, unit="pair-interactions/s", cores=n_all, kind="oracle",
                sample=f"FP64 oracle right-hand sides on {what}, {p_rhs} pairs each: "
                       f"{r_all} on {n_all} threads in {e_all:.1f} s, {r_one} on 1 thread "
                       f"in {e_one:.1f} s",
                value_1thread=v_one, cpu_model=cpu_model(), host_cpus=allt)


def adjoint_bytes(counts, types, prec_bytes, dim):
    """Algorithmic HBM bytes of one reverse right-hand side (sph_rhs_adjoint):
    the forward state and stored derived fields read once per row, the weights
    and seeds read once, the neighbour indices read once per pass that walks
    them (pairs, neighbour average, boundary, density), every adjoint output
    written once. Re-reads of neighbour rows are served by cache and do not
    count."""
    D = dim
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


class Marker:
    """roctx ranges around the timed regions, so that a rocprofv3 trace of this
    command can be restricted to them (--marker-trace). No-op if the roctx
    library is absent."""

    def __init__(self, on):
        self.lib = None
        if on:
            try:
                self.lib = ctypes.CDLL("librocprofiler-sdk-roctx.so")
                self.lib.roctxRangePushA.argtypes = [ctypes.c_char_p]
            except OSError:
                self.lib = None

    def push(self, name):
        if self.lib:
            self.lib.roctxRangePushA(name.encode())

    def pop(self):
        if self.lib:
            self.lib.roctxRangePop()


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


def run_steps(prm, s, prec, args, mark, label):
    """W warm-up steps, then K timed steps between HIP events on the library's
    stream (and the host clock); returns the simulation and its timings."""
    import torch
    from paper_1907_04034_amd import binding as B
    sim = B.Simulation(prm, s, prec=prec)
    stream = torch.cuda.current_stream()
    sim.step(args.warmup)
    bits = sim.poll_error()
    if bits:
        raise SystemExit(f"device error bits after warm-up ({prec}): {bits}")
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    mark.push(f"timed steps {label}")
    w0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    mark.pop()
    gpu_ms = e0.elapsed_time(e1)
    bits = sim.poll_error()
    if bits:
        raise SystemExit(f"device error bits in the timed region ({prec}): {bits}")
    cnt, _ = sim.neighbor_table()
    types = sim.state()["type"]
    p_rhs = int((cnt[types == 0] - 1).sum())
    t_step = max(gpu_ms, wall * 1e3) / args.steps
    log(f"bench {label}: {args.steps} steps in {gpu_ms:.2f} ms (events), {wall * 1e3:.2f} ms "
        f"wall; {p_rhs} pairs per RHS")
    return sim, dict(ms_per_step=t_step, pairs_per_rhs=p_rhs, value=2 * p_rhs / (t_step * 1e-3),
                     n=int(len(types)))


def kernel_timings(sim, prec, args, mark, label):
    """The force pass (sph_force, one kernel launch) and the API's neighbour
    search (sph_neighbor_table with density: the stencil walk, without the
    step path's candidate lists) alone, on a fresh bin of the current state."""
    import torch
    stream = torch.cuda.current_stream()
    sim.bin()
    sim.neighbors()
    sim.rhs()
    torch.cuda.synchronize()
    reps = args.force_reps
    mark.push(f"force launches {label}")
    f_us = 1e3 * timed_launches(stream, reps, lambda: sim.force(reduce_drag=False))
    mark.pop()
    mark.push(f"search launches {label}")
    s_us = 1e3 * timed_launches(stream, max(5, reps // 4), sim.neighbors)
    mark.pop()
    cnt, _ = sim.neighbor_table()
    types = sim.state()["type"]
    if sim.poll_error():
        raise SystemExit(f"device error bits in the kernel timings ({prec})")
    return f_us, s_us, cnt, types


def roofline(prm, prec, f_us, cnt, types, counters):
    import numpy as np
    dim = prm["dim"]
    n = len(types)
    per = SCOPE_BYTES[(dim, prec)][1]
    alg = per * n
    hbm = alg / (f_us * 1e-6) / 1e9
    own = force_bytes(cnt, types, 8 if prec == "fp64" else 4, dim)
    pairs = int((cnt[types == 0] - 1).sum() + np.maximum(cnt[types == 5] - 1, 0).sum())
    flops = FORCE_FLOPS_PER_PAIR * pairs
    tflops = flops / (f_us * 1e-6) / 1e12
    hbm_view = dict(bound="hbm", kernel="k_force", achieved=hbm, peak=HBM_PEAK_GBS,
                    unit="GB/s", frac=hbm / HBM_PEAK_GBS,
                    traffic=(counters or {}).get("traffic"),
                    bytes_per_particle=per, particles=n, algorithmic_bytes_per_launch=alg,
                    launch_us=f_us, own_bytes_per_launch=own,
                    own_achieved_gbs=own / (f_us * 1e-6) / 1e9, source_sha=source_hash())
    alu_view = dict(bound="alu", kernel="k_force", achieved=tflops,
                    peak=VALU_PEAK_TFLOPS[prec], unit="TFLOP/s",
                    frac=tflops / VALU_PEAK_TFLOPS[prec], flops_per_pair=FORCE_FLOPS_PER_PAIR,
                    pairs_per_launch=pairs, launch_us=f_us)
    bound = (counters or {}).get("bound")
    if bound is None:
        bound = "alu" if alu_view["frac"] > hbm_view["frac"] else "hbm"
    main, other = (hbm_view, alu_view) if bound == "hbm" else (alu_view, hbm_view)
    if bound == "alu":
        main["traffic"] = hbm_view["traffic"]
    return main, other


def adjoint_rhs_rate(sim, prec, args, mark):
    """One reverse right-hand side (sph_rhs_adjoint, four kernels) on the
    current state: pair-interactions/s of reversed pairs and its bytes."""
    import numpy as np
    import torch
    stream = torch.cuda.current_stream()
    sim.bin()
    sim.neighbors()
    sim.rhs()
    cnt, _ = sim.neighbor_table()
    types = sim.state()["type"]
    n = len(types)
    rng = np.random.default_rng(0)
    w = rng.standard_normal((n, 3))
    sim.rhs_adjoint(abar=w, bbar=w, pdbar=w[:, 0], fbar=(1.0, 0.0, 0.0))
    torch.cuda.synchronize()
    st = sim._adj_struct((1.0, 0.0, 0.0))
    mark.push("adjoint launches")
    a_us = 1e3 * timed_launches(stream, max(5, args.force_reps // 4),
                                lambda: sim.rhs_adjoint_launch(st))
    mark.pop()
    if sim.poll_error():
        raise SystemExit("device error bits in the adjoint timing")
    p_rhs = int((cnt[types == 0] - 1).sum())
    ab = adjoint_bytes(cnt, types, 8 if prec == "fp64" else 4, sim.dim)
    return dict(value=p_rhs / (a_us * 1e-6), unit="pair-interactions/s", precision=prec,
                launch_us=a_us, pairs_per_rhs=p_rhs, algorithmic_bytes=ab,
                hbm_frac=ab / (a_us * 1e-6) / 1e9 / HBM_PEAK_GBS)


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
    sim2 = B.Simulation(prm, s, prec=args.precision)
    sim2.bin()
    sim2.neighbors()
    sim2.rhs()
    cnt, _ = sim2.neighbor_table()
    types = sim2.state()["type"]
    p_rhs = int((cnt[types == 0] - 1).sum())
    value = 2 * p_rhs * K / (times["backward"] * 1e-3)
    one = adjoint_rhs_rate(sim2, args.precision, args, Marker(False))
    out = {
        "metric": METRIC, "value": value, "unit": "pair-interactions/s", "n_gpus": 1,
        "steps": K, "warmup": min(args.warmup, 20), "ms_per_step": times["backward"] / K,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config] + ", gradient of the time-averaged drag "
                   "w.r.t. the inlet profile", "config": args.config, "form": "adjoint",
                   "particles": int(len(s["p"])), "pairs_per_rhs": p_rhs, "rhs_per_step": 2,
                   "precision": args.precision, "segment": run.segment,
                   "forward_ms": times["forward"], "backward_ms": times["backward"], "J": J},
        "roofline": {"bound": "hbm", "kernel": "sph_rhs_adjoint (4 kernels)",
                     "achieved": one["algorithmic_bytes"] / (one["launch_us"] * 1e-6) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": one["hbm_frac"],
                     "traffic": None, "algorithmic_bytes_per_launch": one["algorithmic_bytes"],
                     "launch_us": one["launch_us"]},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--config", default="C5", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                    help="precision of the line's value")
    ap.add_argument("--forms", default="fp32,adjoint",
                    help="forms timed beside the value (comma list of fp64, fp32, adjoint; "
                         "'none' for none)")
    ap.add_argument("--force-reps", type=int, default=40)
    ap.add_argument("--cpu-budget", type=float, default=10.0,
                    help="seconds of oracle work per thread count (about)")
    ap.add_argument("--cpu-sample-x", type=float, default=0.3,
                    help="3D workloads: the oracle times the particles with x below this")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mark", action="store_true",
                    help="roctx ranges around the timed regions (for rocprofv3 --marker-trace)")
    ap.add_argument("--calibrate-mib", type=int, default=0,
                    help="also run a read-only and a write-only pass over a buffer of this "
                         "size (scales the HBM counters)")
    ap.add_argument("--form", default="forward", choices=["forward", "adjoint"],
                    help="adjoint: gradient of the time-averaged drag (default config C4)")
    ap.add_argument("--segment", type=int, default=50, help="adjoint checkpoint interval")
    ap.add_argument("--outlet", default="hybrid",
                    choices=["hybrid", "moc", "do-nothing", "mod-do-nothing", "mirror"],
                    help="outlet rule (forward form only)")
    ap.add_argument("--mirror-inlet", action="store_true",
                    help="inlet pressure mirrored from the fluid (forward form only)")
    ap.add_argument("--tiles", action="store_true",
                    help="the LDS-tiled neighbour search and force pass instead of the gather "
                         "kernels")
    ap.add_argument("--group-force", type=int, default=0,
                    help="lanes per target of the force pass (1..32; 0: the library's choice)")
    ap.add_argument("--group-nbr", type=int, default=0,
                    help="lanes per target of the neighbour search (1..32; 0: the library's "
                         "choice)")
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
        if "--config" not in sys.argv:
            args.config = "C4"
        if "--steps" not in sys.argv:
            args.steps = 500
        adjoint_bench(args)
        return

    import torch
    from paper_1907_04034_amd import inputs as I

    torch.cuda.set_device(0)
    mark = Marker(args.mark)
    prm, s = I.config(args.config)
    prm["outlet"] = I.OUTLETS[args.outlet]
    prm["group_force"] = args.group_force
    prm["group_nbr"] = args.group_nbr
    if args.mirror_inlet:
        prm["flags"] |= I.FLAG_MIRROR_INLET
    if not args.sort_every_step:
        prm["flags"] |= I.FLAG_REUSE_BINS
    if args.tiles:
        prm["flags"] |= I.FLAG_TILES
    log(f"bench: {prm['name']} n={len(s['p'])} prec={args.precision} "
        f"reuse_bins={not args.sort_every_step} outlet={args.outlet}")

    if args.calibrate_mib:
        nb = args.calibrate_mib << 20
        buf = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
        buf.fill_(1.0)  # write-only: nb bytes
        torch.cuda.synchronize()
        tot = buf.sum()  # read-only: nb bytes
        torch.cuda.synchronize()
        log(f"bench: calibration over {nb} bytes (fill, sum = {float(tot):.0f})")
        del buf

    forms = [f for f in args.forms.split(",") if f and f != "none"]
    sim, main_t = run_steps(prm, s, args.precision, args, mark, args.precision)
    f_us, s_us, cnt, types = kernel_timings(sim, args.precision, args, mark, args.precision)
    counters = counters_summary(args.config, args.precision)
    roof, roof_other = roofline(prm, args.precision, f_us, cnt, types, counters)
    log(f"bench: k_force {f_us:.1f} us/launch ({roof['bound']} {roof['frac']:.3f}), "
        f"stencil search {s_us:.1f} us/launch")
    result_forms = {args.precision: dict(main_t, force_us=f_us, stencil_search_us=s_us,
                                         unit="pair-interactions/s")}
    if "adjoint" in forms:
        result_forms["adjoint"] = adjoint_rhs_rate(sim, args.precision, args, mark)
        log(f"bench: adjoint RHS {result_forms['adjoint']['launch_us']:.1f} us")
    del sim
    torch.cuda.empty_cache()
    for prec in ("fp64", "fp32"):
        if prec in forms and prec != args.precision:
            sim2, t2 = run_steps(prm, s, prec, args, mark, prec)
            f2, s2, c2, ty2 = kernel_timings(sim2, prec, args, mark, prec)
            r2, _ = roofline(prm, prec, f2, c2, ty2, counters_summary(args.config, prec))
            result_forms[prec] = dict(t2, force_us=f2, stencil_search_us=s2, unit="pair-interactions/s",
                                      force_roofline=r2)
            del sim2
            torch.cuda.empty_cache()

    out = {
        "metric": METRIC,
        "value": main_t["value"],
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_t["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "config": args.config,
                   "particles": main_t["n"], "pairs_per_rhs": main_t["pairs_per_rhs"],
                   "rhs_per_step": 2, "precision": args.precision, "outlet": args.outlet,
                   "inlet": "mirror" if args.mirror_inlet else "characteristic",
                   "cell_order": "sorted every step" if args.sort_every_step
                   else "kept while the cell skin allows",
                   "pair_kernels": "LDS tiles" if args.tiles else "gather"},
        "roofline": roof,
        "roofline_other_roof": roof_other,
        "forms": result_forms,
    }
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(prm, s, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
