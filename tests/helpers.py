"""Shared helpers of the GPU parity tests: run the oracle and the HIP path on
the same seeded inputs and measure their differences."""
import numpy as np

from paper_1909_09613_amd import inputs


def oracle_grid(orc, spec):
    return orc.Grid(spec.ndim, spec.n, spec.order, spec.dt, dx=spec.dx, c=spec.c,
                    scheme=spec.scheme, solver=spec.solver)


def copy_species(sp):
    return [{k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in s.items()} for s in sp]


def min_image(d, n):
    """Periodic difference d (cells) mapped into [-n/2, n/2)."""
    return (d + 0.5 * n) % n - 0.5 * n


def particle_errors(spec, ref_sp, got):
    """Max position error (cells) and max relative momentum error over both
    species; got = [(x, u), (x, u)] from the GPU in identity order."""
    ex, eu = 0.0, 0.0
    for s, (x, u) in enumerate(got):
        xr, ur = ref_sp[s]["x"], ref_sp[s]["u"]
        for d in range(spec.ndim):
            ex = max(ex, float(np.max(np.abs(min_image(x[:, d] - xr[:, d], spec.n3[d])))))
        nu = np.linalg.norm(ur, axis=1)
        eu = max(eu, float(np.max(np.linalg.norm(u - ur, axis=1) / np.maximum(nu, 1e-300))))
    return ex, eu


def rel_maxnorm(a, b):
    """||a - b||_inf / ||b||_inf per component (rows)."""
    out = []
    for k in range(a.shape[0]):
        den = np.max(np.abs(b[k]))
        out.append(float(np.max(np.abs(a[k] - b[k])) / den) if den > 0 else float(np.max(np.abs(a[k]))))
    return out


def random_state(spec, seed, amp=0.05, fp32=False):
    """Species and random E, B for a one-step comparison from identical state."""
    sp = inputs.make_species(spec)
    rng = np.random.default_rng(seed)
    E = inputs.random_fields(rng, spec.ncell, amp)
    B = inputs.random_fields(rng, spec.ncell, amp)
    if fp32:
        for s in sp:
            s["x"], s["u"] = inputs.quantize_fp32(s["x"], s["u"])
        E = E.astype(np.float32).astype(np.float64)
        B = B.astype(np.float32).astype(np.float64)
    return sp, E, B


def transverse(spec, k):
    """Current components along a simulated axis other than the drift's:
    driven by the thermal motion only."""
    return k < spec.ndim and k != spec.drift_axis


def abs_current_scale(orc, spec, sp, E, B):
    """Per component, the largest sum over a node of the absolute values of
    the particles' contributions to it (the scale the rounding of a sum is
    measured against).  One particle's contributions to J_k all have the sign
    of Q d_k (its step along k, or Q v_z for J3 in 2D): a prefix sum of
    S1 - S0 along k has one sign for a shift of the form factor, and the
    transverse path averages are >= 0.  So the oracle's current of the
    particles with Q u_k > 0, and that of the rest, give the sum of absolute
    values as |J_k^+| + |J_k^-|."""
    g = oracle_grid(orc, spec)
    g.E[:] = E
    g.B[:] = B
    ref = copy_species(sp)
    for s in ref:
        g.push_species(s["x"], s["u"], s["qm"], s["Q"])
    scale = np.zeros((3, spec.ncell))
    for k in range(3):
        for sign in (1.0, -1.0):
            gk = oracle_grid(orc, spec)
            gk.E[:] = E
            gk.B[:] = B
            gk.zero_J()
            for s, s_new in zip(sp, ref):
                mask = sign * s["Q"] * s_new["u"][:, k] > 0
                if np.any(mask):
                    gk.push_species(s["x"][mask].copy(), s["u"][mask].copy(), s["qm"], s["Q"])
            scale[k] += np.abs(gk.J[k])
    return np.max(scale, axis=1)


def current_tol(spec, k, fp32):
    """Tolerance of J component k against the summed scale.

    FP64: 1e-12 for every component.  The oracle forms S1 - S0 in extended
    precision and the GPU as the step times a divided difference, so both
    keep FP64 relative precision however short the step.

    FP32 (against the sum of absolute contributions, abs_current_scale):
    along the drift (and J3 in 2D) 1e-5.  Transverse components are sums of
    Q * W * d over particles whose transverse steps d are only
    ~ a u_th / gamma0 cells (mean |d| ~ 0.8 a u_th / gamma0 for a Gaussian
    spread); a position error e per particle gives a J error of ~ e / mean|d|
    of the scale, e = 2^-25 cells for the FP32 offset the step is taken from.
    """
    if not fp32:
        return 1e-12
    if not transverse(spec, k):
        return 1e-5
    step = 0.8 * spec.courant * spec.u_th / spec.gamma0
    return max(2e-4, 2.0 ** -25 / step)


def trajectory_vs_oracle(orc, spec, amp, steps, precision, seed=11):
    """`steps` graph-replayed steps (pic_step) of one run from a seeded
    random state with fields of amplitude `amp`, and the same steps of the
    oracle.  Returns the particle position and momentum errors, the E and B
    relative max-norm errors and the number of sorts the device made; asserts
    that no particle was counted non-finite or out of its window."""
    import paper_1909_09613_amd as wt
    fp32 = precision == wt.PIC_MIXED32
    sp, E, B = random_state(spec, seed, amp, fp32=fp32)
    g = oracle_grid(orc, spec)
    g.E[:] = E
    g.B[:] = B
    ref = copy_species(sp)
    sim = wt.Sim([spec], precision)
    try:
        sim.set_species(0, sp)
        sim.set_fields(0, E, B)
        d0 = sim.diagnostics(0)
        sim.step(steps)
        d = sim.diagnostics(0)
        got = [sim.particles(0, s) for s in range(2)]
        Eg, Bg, _ = sim.fields(0)
    finally:
        sim.close()
    for _ in range(steps):
        g.step(ref)
    ex, eu = particle_errors(spec, ref, got)
    eE = max(rel_maxnorm(Eg, g.E))
    eB = max(rel_maxnorm(Bg, g.B))
    print("%dD l=%d %d steps %s: dx=%.2e du=%.2e dE=%.2e dB=%.2e sorts=%d" % (
        spec.ndim, spec.order, steps, "fp32" if fp32 else "fp64", ex, eu, eE, eB, d.n_sorts - d0.n_sorts),
        flush=True)
    assert d.n_nonfinite == 0 and d.n_out_of_range == 0
    return ex, eu, eE, eB, d.n_sorts - d0.n_sorts
