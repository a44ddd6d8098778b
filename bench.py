"""Throughput of the WT gather + push + deposit step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision mixed32|fp64]
                    [--config 2|3|4|5]

Workload (default, --config 2): 2D periodic 1024 x 512 Yee grid,
electron-positron pair plasma drifting along +x1 with gamma 50, thermal
spread u_th = 0.01, 16 particles per cell per species (16.8M particles),
cubic B-spline (l = 3), WT interpolation at c dt = 0.45 dx, synthetic seeded
inputs (the paper's Table 1 recipe at this size).  --config 3, 4, 5 run the
3D 256x128x128 workload, the 64-run batched Courant sweep and the 2D
4096x2048 workload instead.  A step is one full PIC step: re-sort check,
gather + Boris + Esirkepov deposit (one kernel), Yee field update.

Prints one JSON line.  `value` is particle-steps per second of the whole job
over K steps replayed by pic_step from the captured step graph (median of
five repetitions; inputs resident in HBM).  `roofline` refers to the
dominant kernel, the gather-push-deposit kernel: its average launch time is
measured with HIP events recorded by the library on the context stream around
every launch of a separate eager timed region of K steps, and `achieved` is
its algorithmic bytes per
launch (particle state read and written once, E and B read and J written once
per cell) over that time.  `traffic` is the HBM traffic per launch from the
rocprofv3 FETCH_SIZE / WRITE_SIZE counters recorded under profiles/ for the
current kernel source and the default tiling, else null.  `cpu_baseline` is the FP64 CPU oracle
timed on a bounded sample of the same workload on one host core.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published

WORKLOADS = {
    2: "2D periodic 1024x512, drifting pair plasma gamma 50, u_th 0.01, 16 ppc/species, "
       "cubic B-spline, WT at c dt = 0.45 dx",
    3: "3D periodic 256x128x128, drifting pair plasma gamma 50, u_th 0.01, 8 ppc/species, "
       "quadratic B-spline, WT at c dt = 0.5 dx",
    4: "64 batched 2D periodic runs, grids U{128..512} x U{64..256}, c dt/dx = 0.1 + 0.6 r/63, "
       "gamma 10/50/100, u_th 0.01, 8 ppc/species, quadratic B-spline, WT",
    5: "2D periodic 4096x2048, drifting pair plasma gamma 100, u_th 0.01, 16 ppc/species, "
       "cubic B-spline, WT at c dt = 0.3 dx",
}


def particle_bytes(ndim, precision):
    """Bytes of one particle read + written per step."""
    if precision == "fp64":
        return 2 * (8 * ndim + 24)
    return 2 * (4 + 4 * ndim + 12)


def cell_bytes(precision):
    """Bytes per cell per step: E, B read once, FP64 J written once."""
    rs = 8 if precision == "fp64" else 4
    return 6 * rs + 3 * 8


def source_digest():
    """Digest of the particle kernel's sources with comments and blank space
    removed: the stored HBM counters stay valid across comment edits and are
    dropped when code changes."""
    h = hashlib.sha256()
    for name in ("gpd.hip", "common.hpp", "tables.hpp", "runtime.cpp"):
        with open(os.path.join(ROOT, "paper_1909_09613_amd", "csrc", name), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def load_traffic(precision, digest):
    path = os.path.join(ROOT, "profiles", "gpd_traffic_1024x512_l3.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    ent = rec.get(precision)
    if not ent or ent.get("source_digest") != digest:
        return None
    return ent.get("bytes_per_launch")


def cpu_baseline(spec, species, E, B, budget_s=10.0):
    """FP64 oracle (one core) on a bounded sample: the particles of the first
    rows of the grid, pushed for one step at a time until budget_s elapses."""
    from oracle import oracle as orc

    g = orc.Grid(spec.ndim, spec.n, spec.order, spec.dt)
    g.E[:] = E
    g.B[:] = B
    nsample = 65536
    xs = [np.ascontiguousarray(s["x"][:nsample]) for s in species]
    us = [np.ascontiguousarray(s["u"][:nsample]) for s in species]
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        g.zero_J()
        for s, x, u in zip(species, xs, us):
            g.push_species(x, u, s["qm"], s["Q"])
            done += len(x)
    dt = time.perf_counter() - t0
    return {
        "value": done / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
        "sample": "%d particles per species from the first grid rows, %d particle-steps of "
                  "gather+push+deposit (no field update) in %.1f s" % (nsample, done, dt),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--precision", default="mixed32", choices=["mixed32", "fp64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--tile", default=None, help="tile shape, e.g. 32x16")
    ap.add_argument("--margin", type=int, default=0, help="staging margin in cells (0 = default)")
    ap.add_argument("--sort-every", type=int, default=0, help="sort check cadence in steps (0 = default)")
    ap.add_argument("--autotune", type=int, default=0,
                    help="time the library's candidate tilings over this many steps each and keep the "
                         "fastest (0 = the default tiling)")
    ap.add_argument("--config", type=int, default=2, choices=[2, 3, 4, 5], help="workload")
    ap.add_argument("--skip-strip", type=float, default=0.0,
                    help="partially skipped calculation: initially perturbed strip of this width (cells, "
                         "across x1 at the grid centre); 0 = off")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 512 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1909_09613_amd as wt
    from paper_1909_09613_amd import inputs

    specs = inputs.config(args.config)
    spec = specs[0]
    prec = wt.PIC_FP64 if args.precision == "fp64" else wt.PIC_MIXED32
    t_setup = time.perf_counter()
    sim = wt.Sim(specs, prec)
    if args.tile or args.margin or args.sort_every:
        t = ([int(v) for v in args.tile.split("x")] if args.tile else []) + [0, 0, 0]
        wt.pic_set_tiling(sim.ctx, tuple(t[:3]), args.margin, args.sort_every)
    for r, sr in enumerate(specs):
        sim.set_species(r, inputs.make_species(sr))
    if args.skip_strip > 0:
        for r, sr in enumerate(specs):
            mid = 0.5 * sr.n[0]
            sim.set_skip_region(r, (mid - 0.5 * args.skip_strip, 0.0, 0.0),
                                (mid + 0.5 * args.skip_strip, float(sr.n[1]), float(sr.n3[2])), 0.0)
    tuned = None
    if args.autotune > 0:
        tuned = sim.autotune(args.autotune)
        print("autotune: %s" % (tuned,), file=sys.stderr, flush=True)
    np_total = sum(2 * sr.ncell * sr.ppc_s for sr in specs)
    ncell_total = sum(sr.ncell for sr in specs)
    print("setup %.1f s, %d particles" % (time.perf_counter() - t_setup, np_total), file=sys.stderr, flush=True)

    if args.calibrate_copy:
        # a plain copy of known size: 512 MiB read, 512 MiB written
        src = torch.ones(512 * 1024 * 1024 // 4, dtype=torch.float32, device=sim.device)
        dst = torch.empty_like(src)
        with torch.cuda.stream(sim.stream):
            dst.copy_(src)
        sim.synchronize()
        del src, dst

    # the first step sorts every particle (set-up order): timed on its own
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    with torch.cuda.stream(sim.stream):
        start.record(sim.stream)
        sim.gpd()
        stop.record(sim.stream)
    stop.synchronize()
    ms_sort_step = start.elapsed_time(stop)
    sim.field_update()

    # warmup: enough steps that the step graph is captured and replayed at
    # least once before anything is timed
    sim.step(max(args.warmup, 1))
    sim.step(16)
    sim.synchronize()

    # timed region: eager steps with the library's per-launch kernel events
    wt.pic_kernel_timing(sim.ctx, True)
    torch.cuda.synchronize()
    d0 = sim.diagnostics(0)
    with torch.cuda.stream(sim.stream):
        start.record(sim.stream)
        for _ in range(args.steps):
            sim.gpd()
            sim.field_update()
        stop.record(sim.stream)
    stop.synchronize()
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(stop)
    gpd_ms, launches = wt.pic_kernel_timing(sim.ctx, False)

    # the same number of steps replayed from the captured graph, five times;
    # the median is reported
    graph_ms = []
    for _ in range(5):
        torch.cuda.synchronize()
        with torch.cuda.stream(sim.stream):
            start.record(sim.stream)
            sim.step(args.steps)
            stop.record(sim.stream)
        stop.synchronize()
        graph_ms.append(start.elapsed_time(stop))
    ms_graph = float(np.median(graph_ms))

    d = sim.diagnostics(0)
    t_end = d.time
    # one diagnostics call (energies, momentum, Gauss residual) after steps,
    # host clock around the whole call, median of three
    diag_ms = []
    for _ in range(3):
        sim.synchronize()
        t0 = time.perf_counter()
        sim.diagnostics(0)
        diag_ms.append((time.perf_counter() - t0) * 1e3)
    # the field update (a8) alone, after the state above was read: B half
    # step, E step with J, B half step
    torch.cuda.synchronize()
    with torch.cuda.stream(sim.stream):
        start.record(sim.stream)
        for _ in range(args.steps):
            sim.field_update()
        stop.record(sim.stream)
    stop.synchronize()
    field_ms = start.elapsed_time(stop) / args.steps
    sim.close()

    # the step rate: pic_step replays of the captured step graph (the
    # multi-step entry point); the eager region above carries per-launch
    # timing events, whose cache flushes slow each launch by a few percent
    ms_step = ms_graph / args.steps
    value = np_total * args.steps / (ms_graph / 1e3)
    prec_name = args.precision
    alg_bytes = np_total * particle_bytes(spec.ndim, prec_name) + ncell_total * cell_bytes(prec_name)
    achieved = alg_bytes / (gpd_ms / 1e3) / 1e9
    digest = source_digest()
    # the stored counters were taken with the default tiling on this workload
    default_tiling = not (tuned or args.tile or args.margin or args.sort_every)
    traffic = load_traffic(prec_name, digest) if args.config == 2 and default_tiling else None

    if not args.no_cpu:
        rng = np.random.default_rng(0)
        E = inputs.random_fields(rng, spec.ncell, 1e-3)
        B = inputs.random_fields(rng, spec.ncell, 1e-3)
        cpu = cpu_baseline(spec, inputs.make_species(spec), E, B)
        if len(specs) > 1:
            cpu["sample"] += " (first run of the batch)"
    else:
        cpu = None

    out = {
        "metric": "particle-steps/sec (gather+push+deposit) on 1 MI355X; % HBM roofline; FP32 vs FP64",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec_name == "mixed32" else "f64",
        "data": "synthetic",
        "config": {
            "workload": WORKLOADS[args.config],
            "particles": np_total, "precision": prec_name,
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "gpd_kernel", "kernel_ms": gpd_ms, "launches": launches,
            "algorithmic_bytes_per_launch": alg_bytes, "source_digest": digest,
        },
        "graph_repetitions": len(graph_ms),
        "eager_ms_per_step": ms_total / args.steps,
        "breakdown": {
            "gpd_kernel_ms": gpd_ms,
            "rest_of_step_ms": ms_total / args.steps - gpd_ms,
            "field_update_ms": field_ms,
            "first_step_with_full_sort_ms": ms_sort_step,
            "sorts_in_timed_region": d.n_sorts - d0.n_sorts,
            "diagnostics_call_ms": float(np.median(diag_ms)),
        },
        "cpu_baseline": cpu,
        "autotune": tuned,
        "skip": None if args.skip_strip <= 0 else {
            "strip_cells": args.skip_strip,
            "t_end": t_end,
            "perturbed_fraction_at_end": min(1.0, (args.skip_strip + 2 * spec.c * t_end / spec.dx[0]) / spec.n[0]),
            "perturbed_fraction_timed_start": min(1.0, (args.skip_strip + 2 * spec.c * (t_end - spec.dt * args.steps * 6) / spec.dx[0]) / spec.n[0]),
        },
        "check": {"n_nonfinite": d.n_nonfinite, "n_out_of_range": d.n_out_of_range, "n_sorts": d.n_sorts,
                  "field_energy": sum(d.UE) + sum(d.UB)},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
