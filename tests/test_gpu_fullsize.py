"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (default tiling, persistent tile queue), on sampled outputs
the oracle computes one by one:

  * particles: a seeded sample of particle identities per run and species is
    pushed by the oracle (gather + Boris + move) with the same fields and
    compared with the GPU's result for the same identities;
  * current: a few boxes of cells (one straddling the periodic corner); every
    particle that starts within the deposit reach of a box is re-deposited by
    the oracle, per species, which fixes J on the box exactly; the GPU's J on
    the box is compared with the summed-scale metric of the one-step tests;
  * counters: no non-finite value and no particle outside its tile window.

Tolerances are those of the one-step tests (FP64 1e-12; FP32 2e-6, J 1e-5;
transverse J from helpers.current_tol, which scales with the transverse step).  Workloads:
  2D 1024x512, l=3, a=0.45, 16.8M particles (FP32 and FP64);
  3D 256x128x128, l=2, a=0.5, 67.1M particles (FP32 and FP64);
  64 batched 2D runs, l=2, a = 0.1 .. 0.7 (FP32);
  2D 4096x2048, l=3, a=0.3, 268M particles (FP32 and FP64).
"""
import numpy as np
import pytest

import paper_1909_09613_amd as wt
from paper_1909_09613_amd import inputs
from tests import helpers as H

pytestmark = pytest.mark.gpu

AMP = 0.05


def _state(specs, precision, seed):
    fp32 = precision == wt.PIC_MIXED32
    rng = np.random.default_rng(seed)
    sps, fields = [], []
    for spec in specs:
        sp = inputs.make_species(spec)
        E = inputs.random_fields(rng, spec.ncell, AMP)
        B = inputs.random_fields(rng, spec.ncell, AMP)
        if fp32:
            for s in sp:
                s["x"], s["u"] = inputs.quantize_fp32(s["x"], s["u"])
            E = E.astype(np.float32).astype(np.float64)
            B = B.astype(np.float32).astype(np.float64)
        sps.append(sp)
        fields.append((E, B))
    return sps, fields


def _boxes(spec, rng, nbox):
    """Box origins and sizes (cells); the first one straddles the corner."""
    size = (16, 8) if spec.ndim == 2 else (4, 4, 4)
    out = [tuple(n - s // 2 for n, s in zip(spec.n, size))]
    for _ in range(nbox - 1):
        out.append(tuple(int(rng.integers(0, n)) for n in spec.n))
    return [(o, size) for o in out]


def _box_cells(spec, origin, size):
    """Linear indices of the box's cells (periodic)."""
    axes = [(np.arange(s) + o) % n for o, s, n in zip(origin, size, spec.n)]
    grid = np.meshgrid(*axes, indexing="ij")
    lin = grid[0].astype(np.int64)
    stride = 1
    for d in range(1, spec.ndim):
        stride *= spec.n[d - 1]
        lin = lin + stride * grid[d]
    return lin.ravel()


def _in_reach(spec, origin, size, reach):
    """Identities of the particles that start within `reach` cells of the box.
    The generator places particle p in cell p // ppc_s, so these are the
    particles of the cells of the box widened by `reach` on every side."""
    lo, span = [], []
    for o, s, n in zip(origin, size, spec.n):
        whole = s + 2 * reach >= n          # the widened box covers the axis
        lo.append(0 if whole else o - reach)
        span.append(n if whole else s + 2 * reach)
    wide = _box_cells(spec, tuple(lo), tuple(span))
    return (wide[:, None] * spec.ppc_s + np.arange(spec.ppc_s)[None, :]).ravel()


def _check_run(orc, spec, sp, E, B, got, J, precision, nsample, nbox, seed):
    """Sampled particles and boxes of J of one run against the oracle."""
    fp32 = precision == wt.PIC_MIXED32
    rng = np.random.default_rng(seed)
    g = H.oracle_grid(orc, spec)
    g.E[:] = E
    g.B[:] = B
    ex, eu = 0.0, 0.0
    for s in range(2):
        ids = rng.choice(len(sp[s]["x"]), size=min(nsample, len(sp[s]["x"])), replace=False)
        x = sp[s]["x"][ids].copy()
        u = sp[s]["u"][ids].copy()
        g.push_species(x, u, sp[s]["qm"], sp[s]["Q"])
        e1, e2 = H.particle_errors(spec, [{"x": x, "u": u}], [(got[s][0][ids], got[s][1][ids])])
        ex, eu = max(ex, e1), max(eu, e2)
    ej = [0.0, 0.0, 0.0]
    reach = spec.order + 3
    for origin, size in _boxes(spec, rng, nbox):
        cells = _box_cells(spec, origin, size)
        idx = _in_reach(spec, origin, size, reach)
        parts = []
        for s in range(2):
            g.zero_J()
            g.push_species(sp[s]["x"][idx].copy(), sp[s]["u"][idx].copy(), sp[s]["qm"], sp[s]["Q"])
            parts.append(g.J[:, cells].copy())
        ref = parts[0] + parts[1]
        scale = np.max(np.abs(parts[0]) + np.abs(parts[1]), axis=1)
        for k in range(3):
            if scale[k] > 0:
                ej[k] = max(ej[k], float(np.max(np.abs(J[k, cells] - ref[k])) / scale[k]))
    print("fullsize %s %dD %s l=%d a=%.3f: dx=%.2e du=%.2e dJ/scale=%s" % (
        "fp32" if fp32 else "fp64", spec.ndim, "x".join(map(str, spec.n)), spec.order, spec.courant,
        ex, eu, ["%.2e" % v for v in ej]), flush=True)
    if fp32:
        assert ex <= 2e-6 and eu <= 2e-6
        for k in range(3):
            assert ej[k] <= H.current_tol(spec, k, True)
    else:
        assert ex <= 1e-12 and eu <= 1e-12
        for k in range(3):
            assert ej[k] <= H.current_tol(spec, k, False)


def _run(orc, specs, precision, nsample, nbox, seed=5):
    sps, fields = _state(specs, precision, seed)
    sim = wt.Sim(specs, precision)
    try:
        for r in range(len(specs)):
            sim.set_species(r, sps[r])
            sim.set_fields(r, *fields[r])
        sim.gpd()
        for r, spec in enumerate(specs):
            d = sim.diagnostics(r)
            assert d.n_nonfinite == 0 and d.n_out_of_range == 0
            got = [sim.particles(r, s) for s in range(2)]
            _, _, J = sim.fields(r)
            _check_run(orc, spec, sps[r], fields[r][0], fields[r][1], got, J, precision,
                       nsample, nbox, seed + 100 + r)
            del got, J
    finally:
        sim.close()


@pytest.mark.parametrize("precision", [wt.PIC_MIXED32, wt.PIC_FP64], ids=["fp32", "fp64"])
def test_fullsize_2d_1024x512_cubic(orc, precision):
    _run(orc, inputs.config(2), precision, nsample=20000, nbox=6)


@pytest.mark.parametrize("precision", [wt.PIC_MIXED32, wt.PIC_FP64], ids=["fp32", "fp64"])
def test_fullsize_3d_256x128x128(orc, precision):
    _run(orc, inputs.config(3), precision, nsample=4000, nbox=3)


def test_fullsize_batched_courant_sweep(orc):
    _run(orc, inputs.config(4), wt.PIC_MIXED32, nsample=300, nbox=1)


@pytest.mark.parametrize("precision", [wt.PIC_MIXED32, wt.PIC_FP64], ids=["fp32", "fp64"])
def test_fullsize_2d_4096x2048_cubic(orc, precision):
    _run(orc, inputs.config(5), precision, nsample=20000, nbox=4)


def test_fullsize_gauss_law_fp64(orc):
    """Charge conservation at full size: 20 graph-replayed steps of the
    1024x512 drifting plasma keep Gauss's residual at round-off of the
    per-species charge density."""
    spec = inputs.config(2)[0]
    sp = inputs.make_species(spec)
    sim = wt.Sim([spec], wt.PIC_FP64)
    try:
        sim.set_species(0, sp)
        r0 = sim.diagnostics(0).gauss_resid_max
        sim.step(20)
        d = sim.diagnostics(0)
    finally:
        sim.close()
    rho_s = spec.ppc_s * abs(sp[0]["Q"]) / spec.Vc
    print("gauss fullsize: r0=%.3e r20=%.3e rho_s=%.3e" % (r0, d.gauss_resid_max, rho_s), flush=True)
    assert d.n_nonfinite == 0 and d.n_out_of_range == 0
    assert r0 <= 1e-12 * rho_s
    assert d.gauss_resid_max <= 1e-10 * rho_s
