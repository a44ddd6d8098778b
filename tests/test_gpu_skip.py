"""GPU parity of the partially skipped calculation (Sec. 3, "Partially
skipping calculation") against the oracle: outside the region perturbed at
time t (points closer than c t to the box A0) a particle only drifts.

  * one step from identical state with a box whose perturbed region covers
    some tiles completely, misses others and cuts through the rest (the three
    tile classes of the kernel), FP64 and mixed precision, 2D and 3D (with
    anisotropic cells);
  * 20 FP64 steps from t = 0 with the region growing, against the oracle's
    stepping with t = t0 + n dt;
  * two runs in one context, one with the skip and one without, and the skip
    switched off again;
  * argument checks.
Membership is decided in FP64 on both sides; the tests assert that no
particle lies within 1e-9 of the region's boundary, where the two could
legitimately differ by rounding.
"""
import numpy as np
import pytest

import paper_1909_09613_amd as wt
from paper_1909_09613_amd import inputs
from paper_1909_09613_amd.inputs import RunSpec
from tests import helpers as H

pytestmark = pytest.mark.gpu


def _margin_ok(orc, g, sp, lo, hi, t):
    """No particle within 1e-9 (relative) of the boundary of A(t)."""
    for s in sp:
        a = g.perturbed(s["x"], lo, hi, t * (1.0 - 1e-9))
        b = g.perturbed(s["x"], lo, hi, t * (1.0 + 1e-9))
        if np.any(a != b):
            return False
    return True


@pytest.mark.parametrize("precision", [wt.PIC_FP64, wt.PIC_MIXED32], ids=["fp64", "fp32"])
def test_skip_one_step(orc, precision):
    fp32 = precision == wt.PIC_MIXED32
    spec = RunSpec(2, (96, 64), 3, 0.45, 50.0, 0.01, 4, 901)
    sp, E, B = H.random_state(spec, 9, fp32=fp32)
    lo = np.array([40.0, 24.0, 0.0])
    hi = np.array([52.5, 36.0, 0.0])
    t0 = 12.0
    g = H.oracle_grid(orc, spec)
    g.E[:] = E
    g.B[:] = B
    assert _margin_ok(orc, g, sp, lo, hi, t0)
    inside = [g.perturbed(s["x"], lo, hi, t0).astype(bool) for s in sp]
    frac = np.mean(np.concatenate(inside))
    assert 0.1 < frac < 0.6
    # the current per species too: the summed scale of the one-step tests
    # (the two species' currents largely cancel)
    parts = []
    ref = H.copy_species(sp)
    for s in ref:
        g.zero_J()
        g.push_species(s["x"], s["u"], s["qm"], s["Q"], skip=(lo, hi, t0))
        parts.append(g.J.copy())
    sim = wt.Sim([spec], precision)
    try:
        sim.set_species(0, sp)
        sim.set_fields(0, E, B)
        sim.set_skip_region(0, lo, hi, t0)
        sim.gpd()
        got = [sim.particles(0, s) for s in range(2)]
        _, _, J = sim.fields(0)
        d = sim.diagnostics(0)
    finally:
        sim.close()
    assert d.n_nonfinite == 0 and d.n_out_of_range == 0
    for s in range(2):
        # drifting particles keep their momentum bit for bit
        assert np.array_equal(got[s][1][~inside[s]], sp[s]["u"][~inside[s]])
    ex, eu = H.particle_errors(spec, ref, got)
    scale = np.max(np.abs(parts[0]) + np.abs(parts[1]), axis=1)
    ej = [float(np.max(np.abs(J[k] - parts[0][k] - parts[1][k])) / scale[k]) for k in range(3)]
    print("skip one step %s: inside %.2f dx=%.2e du=%.2e dJ=%s" % (
        "fp32" if fp32 else "fp64", frac, ex, eu, ["%.2e" % v for v in ej]), flush=True)
    tol_x = 2e-6 if fp32 else 1e-12
    assert ex <= tol_x and eu <= tol_x
    for k in range(3):
        assert scale[k] > 0
        assert ej[k] <= H.current_tol(spec, k, fp32)


@pytest.mark.parametrize("precision", [wt.PIC_FP64, wt.PIC_MIXED32], ids=["fp64", "fp32"])
def test_skip_one_step_3d(orc, precision):
    """3D with anisotropic cells: the distance is Euclidean in physical units."""
    fp32 = precision == wt.PIC_MIXED32
    spec = RunSpec(3, (32, 24, 20), 2, 0.4, 50.0, 0.01, 2, 906, dx=(1.0, 0.8, 1.25))
    sp, E, B = H.random_state(spec, 10, fp32=fp32)
    lo = np.array([12.0, 8.0, 6.0])
    hi = np.array([16.0, 12.5, 9.0])
    t0 = 5.0
    g = H.oracle_grid(orc, spec)
    g.E[:] = E
    g.B[:] = B
    assert _margin_ok(orc, g, sp, lo, hi, t0)
    inside = [g.perturbed(s["x"], lo, hi, t0).astype(bool) for s in sp]
    frac = np.mean(np.concatenate(inside))
    assert 0.1 < frac < 0.7
    parts = []
    ref = H.copy_species(sp)
    for s in ref:
        g.zero_J()
        g.push_species(s["x"], s["u"], s["qm"], s["Q"], skip=(lo, hi, t0))
        parts.append(g.J.copy())
    sim = wt.Sim([spec], precision)
    try:
        sim.set_species(0, sp)
        sim.set_fields(0, E, B)
        sim.set_skip_region(0, lo, hi, t0)
        sim.gpd()
        got = [sim.particles(0, s) for s in range(2)]
        _, _, J = sim.fields(0)
        d = sim.diagnostics(0)
    finally:
        sim.close()
    assert d.n_nonfinite == 0 and d.n_out_of_range == 0
    for s in range(2):
        assert np.array_equal(got[s][1][~inside[s]], sp[s]["u"][~inside[s]])
    ex, eu = H.particle_errors(spec, ref, got)
    scale = np.max(np.abs(parts[0]) + np.abs(parts[1]), axis=1)
    ej = [float(np.max(np.abs(J[k] - parts[0][k] - parts[1][k])) / scale[k]) for k in range(3)]
    print("skip one step 3D %s: inside %.2f dx=%.2e du=%.2e dJ=%s" % (
        "fp32" if fp32 else "fp64", frac, ex, eu, ["%.2e" % v for v in ej]), flush=True)
    tol_x = 2e-6 if fp32 else 1e-12
    assert ex <= tol_x and eu <= tol_x
    for k in range(3):
        assert ej[k] <= H.current_tol(spec, k, fp32)


def test_skip_trajectory_fp64(orc):
    spec = RunSpec(2, (64, 48), 2, 0.5, 20.0, 0.05, 2, 902)
    sp = inputs.make_species(spec)
    lo = np.array([28.0, 20.0, 0.0])
    hi = np.array([36.0, 28.0, 0.0])
    g = H.oracle_grid(orc, spec)
    ref = H.copy_species(sp)
    nsteps = 20
    for n in range(nsteps):
        t = 0.0 + n * spec.dt
        assert _margin_ok(orc, g, ref, lo, hi, t)
        g.step(ref, skip=(lo, hi, t))
    sim = wt.Sim([spec], wt.PIC_FP64)
    try:
        sim.set_species(0, sp)
        sim.set_skip_region(0, lo, hi, 0.0)
        for _ in range(nsteps):
            sim.gpd()
            sim.field_update()
        got = [sim.particles(0, s) for s in range(2)]
        Eg, Bg, _ = sim.fields(0)
    finally:
        sim.close()
    # the same steps replayed from the step graph (the region's time is kept
    # on the device)
    sim = wt.Sim([spec], wt.PIC_FP64)
    try:
        sim.set_species(0, sp)
        sim.set_skip_region(0, lo, hi, 0.0)
        sim.step(nsteps)
        got_g = [sim.particles(0, s) for s in range(2)]
    finally:
        sim.close()
    exg, eug = H.particle_errors(spec, ref, got_g)
    assert exg <= 1e-10 and eug <= 1e-10
    ex, eu = H.particle_errors(spec, ref, got)
    eE = H.rel_maxnorm(Eg, g.E)
    eB = H.rel_maxnorm(Bg, g.B)
    print("skip trajectory: dx=%.2e du=%.2e dE=%s dB=%s" % (ex, eu, eE, eB), flush=True)
    assert ex <= 1e-10 and eu <= 1e-10
    assert max(eE) <= 1e-9 and max(eB) <= 1e-9
    # far from the box the momenta are the loaded ones
    inside = [g.perturbed(s["x"], lo, hi, nsteps * spec.dt) for s in ref]
    for s in range(2):
        far = inside[s] == 0
        assert far.sum() > 100
        assert np.array_equal(got[s][1][far], sp[s]["u"][far])


def test_skip_per_run_and_switched_off(orc):
    """Run 0 skips, run 1 of the same context does not; then the skip is
    switched off for run 0 and a step matches the plain step."""
    s0 = RunSpec(2, (48, 32), 2, 0.45, 50.0, 0.01, 2, 903)
    s1 = RunSpec(2, (40, 24), 2, 0.3, 10.0, 0.01, 2, 904)
    lo = np.array([20.0, 12.0, 0.0])
    hi = np.array([26.0, 18.0, 0.0])
    t0 = 5.0
    sps = [inputs.make_species(s0), inputs.make_species(s1)]
    sim = wt.Sim([s0, s1], wt.PIC_FP64)
    try:
        for r in range(2):
            sim.set_species(r, sps[r])
        sim.set_skip_region(0, lo, hi, t0)
        sim.gpd()
        got = [[sim.particles(r, s) for s in range(2)] for r in range(2)]
        _, _, J0 = sim.fields(0)
        _, _, J1 = sim.fields(1)
        sim.field_update()
        sim.set_skip_region(0, None)
        mid = [sim.particles(0, s) for s in range(2)]
        E0, B0, _ = sim.fields(0)
        sim.gpd()
        after = [sim.particles(0, s) for s in range(2)]
    finally:
        sim.close()
    for r, spec in enumerate((s0, s1)):
        g = H.oracle_grid(orc, spec)
        ref = H.copy_species(sps[r])
        for s in ref:
            g.push_species(s["x"], s["u"], s["qm"], s["Q"], skip=(lo, hi, t0) if r == 0 else None)
        ex, eu = H.particle_errors(spec, ref, got[r])
        Jg = J0 if r == 0 else J1
        # against the scale of either species' current (they largely cancel)
        jmax = np.max(np.abs(g.J), axis=1)
        q = abs(spec.species_constants()[0][1])
        jscale = 2 * spec.ppc_s * q * spec.c / spec.Vc
        assert ex <= 1e-12 and eu <= 1e-12, r
        assert np.max(np.abs(Jg - g.J)) <= 1e-12 * max(jscale, np.max(jmax)), r
    # with the skip off the next step is the plain step from the same state
    g = H.oracle_grid(orc, s0)
    g.E[:] = E0
    g.B[:] = B0
    ref = H.copy_species(sps[0])
    for s in range(2):
        ref[s]["x"], ref[s]["u"] = mid[s][0].copy(), mid[s][1].copy()
        g.push_species(ref[s]["x"], ref[s]["u"], ref[s]["qm"], ref[s]["Q"])
    ex, eu = H.particle_errors(s0, ref, after)
    assert ex <= 1e-12 and eu <= 1e-12


def test_skip_region_arguments(orc):
    spec = RunSpec(2, (24, 16), 1, 0.4, 5.0, 0.01, 1, 905)
    sim = wt.Sim([spec], wt.PIC_MIXED32)
    try:
        for lo, hi, t0 in (((-1.0, 0.0), (2.0, 2.0), 0.0), ((3.0, 0.0), (2.0, 2.0), 0.0),
                           ((0.0, 0.0), (25.0, 2.0), 0.0), ((0.0, 0.0), (2.0, 2.0), -1.0),
                           ((0.0, 0.0), (np.nan, 2.0), 0.0)):
            with pytest.raises(wt.PicError) as e:
                sim.set_skip_region(0, lo, hi, t0)
            assert e.value.status == wt.PIC_ERR_ARG
        with pytest.raises(wt.PicError):
            sim.set_skip_region(1, (0.0, 0.0), (1.0, 1.0), 0.0)
        sim.set_skip_region(0, (0.0, 0.0), (24.0, 16.0), 0.0)
        sim.set_skip_region(0, None)
    finally:
        sim.close()
