"""Throughput of the WT gather + push + deposit step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2|3|4|5]
                    [--precision both|mixed32|fp64] [--no-cpu] [--no-check]

Workload (default, --config 5): 2D periodic 4096 x 2048 Yee grid,
electron-positron pair plasma drifting along +x1 with gamma 100, thermal
spread u_th = 0.01, 16 particles per cell per species (268M particles), cubic
B-spline (l = 3), WT interpolation at c dt = 0.3 dx, synthetic seeded inputs
(the paper's Table 1 recipe at this size).  --config 2, 3, 4 run the 2D
1024x512 workload, the 3D 256x128x128 workload and the 64-run batched Courant
sweep instead.  A step is one full PIC step: re-sort check, gather + Boris +
Esirkepov deposit (one kernel), Yee field update.

Prints one JSON line.  `value` is the mixed-precision (FP32 particle state,
FP64 current) path's particle-steps per second of the whole job over K steps
replayed by pic_step from the captured step graph (median of five
repetitions; inputs resident in HBM); `fp64` holds the same figures for the
FP64 path, measured in the same run.  `roofline` refers to the dominant
kernel, the gather-push-deposit kernel: its average launch time comes from
HIP events on the context stream around a graph holding that kernel alone,
replayed once per step of K further steps after W discarded ones
(pic_kernel_timing; the sort checks and the field update run between the
replays), and `achieved` is its algorithmic
bytes per launch (particle state read and written once, E and B read and J
written once per cell) over that time.  `traffic` is the HBM traffic per
launch from rocprofv3 FETCH_SIZE / WRITE_SIZE counters stored under profiles/
for the current kernel source, workload and default tiling, else null;
`valu` is the vector-instruction issue rate from the stored SQ_INSTS_VALU
count over the same launch time, against one wave-instruction per clock per
CU.

The CPU-baseline leg is the only part that runs the FP64 CPU oracle: it times
it on a bounded sample of the workload, on one core and on all host cores
(one process per core on disjoint samples), and it pushes sampled particles of
the workload one step from the state the GPU legs stepped, so that the line
carries the GPU path's error against the oracle for each precision.
"""
import argparse
import hashlib
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
CUS, CLOCK_GHZ = 256, 2.4      # MI355X compute units and peak engine clock
CHECK_AMP = 0.05               # field amplitude of the one-step check against the oracle

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
COUNTER_KEYS = {2: "2d_1024x512_l3", 3: "3d_256x128x128_l2", 4: "2d_batched64_l2", 5: "2d_4096x2048_l3"}


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
    removed: stored counters stay valid across comment edits and are dropped
    when code changes."""
    h = hashlib.sha256()
    for name in ("gpd.hip", "common.hpp", "tables.hpp", "runtime.cpp"):
        with open(os.path.join(ROOT, "paper_1909_09613_amd", "csrc", name), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def load_counters(config, precision, digest):
    """Stored rocprofv3 counters of the particle kernel (per launch) for this
    workload and precision, if they were taken from the current source."""
    path = os.path.join(ROOT, "profiles", "gpd_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    ent = rec.get(COUNTER_KEYS[config], {}).get(precision)
    if not ent or ent.get("source_digest") != digest:
        return None
    return ent


# ---- the CPU-baseline leg (the only code here that runs the oracle) ---------

def _patch_spec(spec, rows, seed_shift):
    """A periodic patch of the workload: the same order, Courant number,
    drift, thermal spread and particles per cell on n0' x rows cells."""
    from paper_1909_09613_amd.inputs import RunSpec

    n = list(spec.n)
    n[0] = min(n[0], 256 if spec.ndim == 2 else 32)
    for d in range(1, spec.ndim):
        n[d] = min(n[d], rows)
    return RunSpec(spec.ndim, tuple(n), spec.order, spec.courant, spec.gamma0, spec.u_th, spec.ppc_s,
                   spec.seed + 7919 * seed_shift, scheme=spec.scheme, solver=spec.solver,
                   skin_depth_cells=spec.skin_depth_cells, dx=spec.dx, c=spec.c, drift_axis=spec.drift_axis)


def _oracle_rate(spec, budget_s):
    """Whole gather+push+deposit steps of the oracle over a patch's particles
    until budget_s elapses; returns (particle-steps, seconds)."""
    from oracle import oracle as orc
    from paper_1909_09613_amd import inputs

    sp = inputs.make_species(spec, workers=1)
    g = orc.Grid(spec.ndim, spec.n, spec.order, spec.dt, dx=spec.dx, c=spec.c, scheme=spec.scheme,
                 solver=spec.solver)
    rng = np.random.default_rng(spec.seed)
    g.E[:] = inputs.random_fields(rng, spec.ncell, 1e-3)
    g.B[:] = inputs.random_fields(rng, spec.ncell, 1e-3)
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        g.zero_J()
        for s in sp:
            g.push_species(s["x"], s["u"], s["qm"], s["Q"])
            done += len(s["x"])
    return done, time.perf_counter() - t0


def cpu_worker(arg):
    """Entry of one all-core worker process: prints its (particle-steps, s)."""
    spec_kw = json.loads(arg)
    from paper_1909_09613_amd.inputs import RunSpec

    spec = RunSpec(**{k: tuple(v) if isinstance(v, list) else v for k, v in spec_kw["spec"].items()})
    done, dt = _oracle_rate(spec, spec_kw["budget"])
    print(json.dumps({"done": done, "seconds": dt}), flush=True)


def host_cores():
    """Cores this process may run on, capped at the 16 a one-GPU machine grants."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(spec, budget_s=10.0):
    """The oracle on one core, then on every host core at once (one process
    per core, each on its own patch), over patches of the workload."""
    import dataclasses

    rows = 16 if spec.ndim == 2 else 8
    one = _patch_spec(spec, rows, 0)
    done, dt = _oracle_rate(one, budget_s)
    single = {"value": done / dt, "cores": 1, "particle_steps": done, "seconds": dt}
    ncores = host_cores()
    procs = []
    for k in range(ncores):
        kw = dataclasses.asdict(_patch_spec(spec, rows, k + 1))
        arg = json.dumps({"spec": kw, "budget": budget_s})
        procs.append(subprocess.Popen([sys.executable, os.path.abspath(__file__), "--cpu-worker", arg],
                                      stdout=subprocess.PIPE, text=True))
    total, tmax = 0, 0.0
    for p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("CPU baseline worker failed")
        r = json.loads(out.strip().splitlines()[-1])
        total += r["done"]
        tmax = max(tmax, r["seconds"])
    patch = "x".join(str(v) for v in one.n)
    return {
        "value": total / tmax, "unit": "particle-steps/s", "cores": ncores, "kind": "oracle",
        "sample": "%d processes, each a %s-cell periodic patch of the workload (same order, Courant number, "
                  "drift, spread, particles per cell; %d particles) pushed whole gather+push+deposit steps "
                  "for ~%.0f s; %d particle-steps in %.1f s" % (ncores, patch, 2 * one.ncell * one.ppc_s,
                                                                  budget_s, total, tmax),
        "single_core": single,
    }


def oracle_errors(specs, runs_checked, species, fields, got, precision, nsample=4000):
    """One step of the oracle from the state the GPU stepped (its fields
    and the sampled particles) against the GPU's result: max position error
    (cells), max relative momentum error, and J on a box (every particle that
    starts within the deposit reach re-deposited) against the summed scale of
    both species, per component."""
    from oracle import oracle as orc

    ex = eu = 0.0
    ej = [0.0, 0.0, 0.0]
    for r in runs_checked:
        spec = specs[r]
        E, B = fields[r]
        g = orc.Grid(spec.ndim, spec.n, spec.order, spec.dt, dx=spec.dx, c=spec.c, scheme=spec.scheme,
                     solver=spec.solver)
        g.E[:] = E
        g.B[:] = B
        rng = np.random.default_rng(100 + r)
        (xg0, ug0), (xg1, ug1), Jg = got[r]
        for s, (xg, ug) in enumerate(((xg0, ug0), (xg1, ug1))):
            sp = species[r][s]
            ids = rng.choice(len(sp["x"]), size=min(nsample, len(sp["x"])), replace=False)
            x = sp["x"][ids].copy()
            u = sp["u"][ids].copy()
            g.push_species(x, u, sp["qm"], sp["Q"])
            for d in range(spec.ndim):
                dd = (xg[ids, d] - x[:, d] + 0.5 * spec.n3[d]) % spec.n3[d] - 0.5 * spec.n3[d]
                ex = max(ex, float(np.max(np.abs(dd))))
            eu = max(eu, float(np.max(np.linalg.norm(ug[ids] - u, axis=1) / np.linalg.norm(u, axis=1))))
        # a box of cells at a random place; the generator puts particle p in
        # cell p // ppc_s, so the particles within reach are those of the
        # widened box's cells
        size = (16, 8) if spec.ndim == 2 else (4, 4, 4)
        reach = spec.order + 3
        origin = [int(rng.integers(0, n)) for n in spec.n]
        axes = [(np.arange(sz) + o) % n for o, sz, n in zip(origin, size, spec.n)]
        wide = [(np.arange(sz + 2 * reach) + o - reach) % n for o, sz, n in zip(origin, size, spec.n)]

        def lin(ax):
            m = np.meshgrid(*ax, indexing="ij")
            out = m[0].astype(np.int64)
            stride = 1
            for d in range(1, spec.ndim):
                stride *= spec.n[d - 1]
                out = out + stride * m[d]
            return out.ravel()

        cells = lin(axes)
        idx = (np.unique(lin(wide))[:, None] * spec.ppc_s + np.arange(spec.ppc_s)[None, :]).ravel()
        parts = []
        for s in range(2):
            sp = species[r][s]
            g.zero_J()
            g.push_species(sp["x"][idx].copy(), sp["u"][idx].copy(), sp["qm"], sp["Q"])
            parts.append(g.J[:, cells].copy())
        scale = np.max(np.abs(parts[0]) + np.abs(parts[1]), axis=1)
        for k in range(3):
            if scale[k] > 0:
                ej[k] = max(ej[k], float(np.max(np.abs(Jg[k, cells] - (parts[0][k] + parts[1][k]))) / scale[k]))
    return {"position_cells": ex, "momentum_rel": eu, "J_rel_summed_scale": ej,
            "sample": "%d particles per species and a %s-cell box of J per checked run (runs %s), one step "
                      "from seeded fields of amplitude %g" % (nsample, "x".join(map(str, size)),
                                                              list(runs_checked), CHECK_AMP)}


# ---- the GPU legs -------------------------------------------------------------

def run_leg(args, specs, species, prec_name, check_runs):
    """Everything measured for one precision: the one-step state the oracle
    is compared with, the first (fully sorting) step, the graph-replayed step
    rate, the graph-replayed particle-kernel time, the field update alone."""
    import torch

    import paper_1909_09613_amd as wt
    from paper_1909_09613_amd import inputs

    prec = wt.PIC_FP64 if prec_name == "fp64" else wt.PIC_MIXED32
    fp32 = prec == wt.PIC_MIXED32
    sim = wt.Sim(specs, prec)
    out = {}
    try:
        if args.tile or args.margin or args.sort_every:
            t = ([int(v) for v in args.tile.split("x")] if args.tile else []) + [0, 0, 0]
            wt.pic_set_tiling(sim.ctx, tuple(t[:3]), args.margin, args.sort_every)
        sp_used = species
        if fp32:
            # the FP32 layout holds exactly these values; the oracle then
            # starts from the same state
            sp_used = []
            for sps in species:
                q = []
                for s in sps:
                    x, u = inputs.quantize_fp32(s["x"], s["u"])
                    q.append(dict(s, x=x, u=u))
                sp_used.append(q)
        for r in range(len(specs)):
            sim.set_species(r, sp_used[r])
        check = None
        if not args.no_check:
            rng = np.random.default_rng(77)
            fields = {}
            for r in check_runs:
                E = inputs.random_fields(rng, specs[r].ncell, CHECK_AMP)
                B = inputs.random_fields(rng, specs[r].ncell, CHECK_AMP)
                if fp32:
                    E = E.astype(np.float32).astype(np.float64)
                    B = B.astype(np.float32).astype(np.float64)
                fields[r] = (E, B)
                sim.set_fields(r, E, B)
            sim.gpd()
            got = {r: (sim.particles(r, 0), sim.particles(r, 1), sim.fields(r)[2]) for r in check_runs}
            check = (fields, got, sp_used)
            # back to the workload's initial state: particles as loaded, no fields
            for r in range(len(specs)):
                sim.set_species(r, sp_used[r])
                z = np.zeros((3, specs[r].ncell))
                sim.set_fields(r, z, z)
        if args.skip_strip > 0:
            for r, sr in enumerate(specs):
                mid = 0.5 * sr.n[0]
                sim.set_skip_region(r, (mid - 0.5 * args.skip_strip, 0.0, 0.0),
                                    (mid + 0.5 * args.skip_strip, float(sr.n[1]), float(sr.n3[2])), 0.0)
        tuned = None
        if args.autotune > 0:
            tuned = sim.autotune(args.autotune)
            print("autotune %s: %s" % (prec_name, tuned), file=sys.stderr, flush=True)

        if args.calibrate_copy:
            # a plain copy of known size: 512 MiB read, 512 MiB written
            src = torch.ones(512 * 1024 * 1024 // 4, dtype=torch.float32, device=sim.device)
            dst = torch.empty_like(src)
            with torch.cuda.stream(sim.stream):
                dst.copy_(src)
            sim.synchronize()
            del src, dst

        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        # the first step sorts every particle (set-up order): timed on its own
        torch.cuda.synchronize()
        with torch.cuda.stream(sim.stream):
            start.record(sim.stream)
            sim.gpd()
            stop.record(sim.stream)
        stop.synchronize()
        ms_sort_step = start.elapsed_time(stop)
        sim.field_update()
        # warmup: enough steps that the step graph is captured and replayed
        sim.step(max(args.warmup, 1))
        sim.step(16)
        sim.synchronize()
        d0 = sim.diagnostics(0)

        # the step rate: K steps replayed from the captured step graph, five
        # times; the median is reported
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

        # the particle kernel's own time: K more steps, each replaying a graph
        # of the particle kernel alone between two stream events, after W
        # steps in the same mode whose times are discarded (the first launches
        # of the switched mode run slower)
        wt.pic_kernel_timing(sim.ctx, True)
        sim.step(max(args.warmup, 3))
        wt.pic_kernel_timing(sim.ctx, True)
        sim.step(args.steps)
        gpd_ms, launches = wt.pic_kernel_timing(sim.ctx, False)

        d = sim.diagnostics(0)
        t_end = d.time
        diag_ms = []
        for _ in range(3):
            sim.synchronize()
            t0 = time.perf_counter()
            sim.diagnostics(0)
            diag_ms.append((time.perf_counter() - t0) * 1e3)
        # the field update (B half step, E step with J, B half step) alone
        torch.cuda.synchronize()
        with torch.cuda.stream(sim.stream):
            start.record(sim.stream)
            for _ in range(args.steps):
                sim.field_update()
            stop.record(sim.stream)
        stop.synchronize()
        field_ms = start.elapsed_time(stop) / args.steps
    finally:
        sim.close()
        del sim
        torch.cuda.empty_cache()

    np_total = sum(2 * sr.ncell * sr.ppc_s for sr in specs)
    ncell_total = sum(sr.ncell for sr in specs)
    ms_step = ms_graph / args.steps
    alg_bytes = np_total * particle_bytes(specs[0].ndim, prec_name) + ncell_total * cell_bytes(prec_name)
    achieved = alg_bytes / (gpd_ms / 1e3) / 1e9
    digest = source_digest()
    default_tiling = not (tuned or args.tile or args.margin or args.sort_every or args.skip_strip > 0)
    ctr = load_counters(args.config, prec_name, digest) if default_tiling else None
    valu = None
    traffic = None
    if ctr:
        traffic = ctr.get("hbm_bytes_per_launch")
        if ctr.get("valu_insts_per_launch"):
            rate = ctr["valu_insts_per_launch"] / (gpd_ms / 1e3)
            peak = CUS * CLOCK_GHZ * 1e9
            valu = {"insts_per_launch": ctr["valu_insts_per_launch"], "achieved": rate, "peak": peak,
                    "unit": "wave-instructions/s", "frac": rate / peak,
                    # a wave-instruction serves 64 particles, one per lane: this is
                    # the count of vector instructions each particle goes through
                    "per_particle_lane": ctr["valu_insts_per_launch"] * 64.0 / np_total}
    out.update({
        "value": np_total * args.steps / (ms_graph / 1e3),
        "ms_per_step": ms_step,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "valu": valu,
            "kernel": "gpd_kernel", "kernel_ms": gpd_ms, "launches": launches,
            "kernel_timing": "HIP events around a one-kernel graph replayed once per step",
            "algorithmic_bytes_per_launch": alg_bytes, "source_digest": digest,
        },
        "graph_repetitions": len(graph_ms),
        "breakdown": {
            "gpd_kernel_ms": gpd_ms,
            "rest_of_step_ms": ms_step - gpd_ms,
            "field_update_ms": field_ms,
            "first_step_with_full_sort_ms": ms_sort_step,
            "sorts_in_timed_region": d.n_sorts - d0.n_sorts,
            "diagnostics_call_ms": float(np.median(diag_ms)),
        },
        "autotune": tuned,
        "skip": None if args.skip_strip <= 0 else {
            "strip_cells": args.skip_strip, "t_end": t_end,
            "perturbed_fraction_at_end": min(1.0, (args.skip_strip + 2 * specs[0].c * t_end / specs[0].dx[0])
                                             / specs[0].n[0]),
        },
        "state_check": {"n_nonfinite": d.n_nonfinite, "n_out_of_range": d.n_out_of_range, "n_sorts": d.n_sorts,
                        "field_energy": sum(d.UE) + sum(d.UB)},
    })
    return out, check


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--precision", default="both", choices=["both", "mixed32", "fp64"])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-check", action="store_true", help="skip the one-step error against the oracle")
    ap.add_argument("--tile", default=None, help="tile shape, e.g. 32x16")
    ap.add_argument("--margin", type=int, default=0, help="staging margin in cells (0 = default)")
    ap.add_argument("--sort-every", type=int, default=0, help="sort check cadence in steps (0 = default)")
    ap.add_argument("--autotune", type=int, default=0,
                    help="time the library's candidate tilings over this many steps each and keep the "
                         "fastest (0 = the default tiling)")
    ap.add_argument("--config", type=int, default=5, choices=[2, 3, 4, 5], help="workload")
    ap.add_argument("--skip-strip", type=float, default=0.0,
                    help="partially skipped calculation: initially perturbed strip of this width (cells, "
                         "across x1 at the grid centre); 0 = off")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run one plain 512 MiB device copy (HBM counter calibration)")
    ap.add_argument("--cpu-worker", default=None, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker is not None:
        cpu_worker(args.cpu_worker)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(got --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    from paper_1909_09613_amd import inputs

    specs = inputs.config(args.config)
    spec = specs[0]
    # the CPU baseline runs first, before anything touches the GPU
    cpu = None
    if not args.no_cpu:
        t0 = time.perf_counter()
        cpu = cpu_baseline(spec)
        if len(specs) > 1:
            cpu["sample"] += " (patches of the first run of the batch)"
        print("cpu baseline %.1f s" % (time.perf_counter() - t0), file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    species = [inputs.make_species(sr) for sr in specs]
    np_total = sum(2 * sr.ncell * sr.ppc_s for sr in specs)
    print("inputs %.1f s, %d particles" % (time.perf_counter() - t0, np_total), file=sys.stderr, flush=True)
    check_runs = [0] if len(specs) == 1 else [0, len(specs) // 3, 42 % len(specs), len(specs) - 1]
    precs = ["mixed32", "fp64"] if args.precision == "both" else [args.precision]
    legs, checks = {}, {}
    for p in precs:
        t0 = time.perf_counter()
        legs[p], checks[p] = run_leg(args, specs, species, p, check_runs)
        print("%s leg %.1f s: %.4g particle-steps/s, %.4f ms/step, kernel %.4f ms" % (
            p, time.perf_counter() - t0, legs[p]["value"], legs[p]["ms_per_step"],
            legs[p]["roofline"]["kernel_ms"]), file=sys.stderr, flush=True)

    # CPU-baseline leg, second part: the oracle's step of the same sampled
    # particles from the state each GPU leg stepped
    errors = None
    if not args.no_check:
        errors = {}
        for p in precs:
            fields, got, sp_used = checks[p]
            errors[p] = oracle_errors(specs, check_runs, sp_used, fields, got, p)
        del checks

    head = legs[precs[0]]
    out = {
        "metric": "particle-steps/sec (gather+push+deposit) on 1 MI355X; % HBM roofline; FP32 vs FP64",
        "value": head["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if precs[0] == "mixed32" else "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.config], "particles": np_total, "precision": precs[0]},
        "roofline": head["roofline"],
        "graph_repetitions": head["graph_repetitions"],
        "breakdown": head["breakdown"],
    }
    if len(precs) > 1:
        other = legs[precs[1]]
        out[precs[1]] = {
            "value": other["value"], "ms_per_step": other["ms_per_step"], "dtype": "f64",
            "frac": other["roofline"]["frac"], "roofline": other["roofline"], "breakdown": other["breakdown"],
            "state_check": other["state_check"],
        }
    out["error_vs_oracle"] = errors
    out["cpu_baseline"] = cpu
    out["autotune"] = {p: legs[p]["autotune"] for p in precs} if args.autotune > 0 else None
    out["skip"] = head["skip"]
    out["state_check"] = head["state_check"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
