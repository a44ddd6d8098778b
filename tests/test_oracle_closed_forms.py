"""Closed-form pins of oracle parts that the kernel and continuity pins do not
reach on their own:

  * the relativistic Boris push with E and B acting together (Sec. 1 names
    the push): removing the two half electric kicks must leave a pure
    rotation about B, by the Boris angle 2 atan(|eps| |B| / gamma^-) taken at
    the gamma of the half-kicked momentum;
  * the out-of-plane current of the 2D deposit (Sec. 1 and 2, Esirkepov's
    decomposition): a 3D path that moves by v_z dt along x3 carries, summed
    over the x3 nodes, exactly the 2D J3 of the same (x1, x2) path;
  * the energy sums of the Sec. 4 observable: a single cosine mode of
    amplitude A on N cells of volume Vc holds 1/2 A^2 (N/2) Vc, and the
    kinetic energy of momenta with integer gamma is M sum (gamma - 1) c^2;
  * the fourth-order dispersion of the M4 Faraday stencil (Appendix C): the
    phase-velocity error of a vacuum mode, with the phase taken from the
    oracle's own leapfrog, falls 16-fold when k halves (4-fold for Yee).
"""
import numpy as np
import pytest


# ---------------------------------------------------------------------------
# Boris with E and B together
# ---------------------------------------------------------------------------

def _boris_cases(seed, n):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        u = rng.normal(size=3) * rng.choice([0.1, 3.0, 60.0])
        E = rng.normal(size=3) * rng.choice([0.01, 1.0, 20.0])
        B = rng.normal(size=3) * rng.choice([0.01, 1.0, 20.0])
        qm = float(rng.choice([-1.0, 1.0])) * rng.uniform(0.5, 2.0)
        dt = rng.uniform(0.05, 0.9)
        c = float(rng.choice([1.0, 1.7]))
        yield u, E, B, qm, dt, c


def test_boris_e_and_b_kick_rotate_kick(orc):
    """u^- = u + eps E and u^+ = u_out - eps E (eps = (q/m) dt / (2c)) have
    the same length, the same component along B, and their components
    across B differ by a rotation about B of -sign(q) 2 atan(|eps| |B| /
    gamma^-), gamma^- = sqrt(1 + |u^-|^2).  A push that takes gamma from
    u^{n-1/2}, or applies the electric kick on one side of the rotation only,
    breaks one of these."""
    for u, E, B, qm, dt, c in _boris_cases(5, 200):
        eps = qm * dt / (2.0 * c)
        out = orc.boris(u, E, B, qm, dt, c)
        um = u + eps * E
        up = out - eps * E
        nm = np.linalg.norm(um)
        assert abs(np.linalg.norm(up) - nm) <= 2e-15 * max(nm, 1.0)
        bh = B / np.linalg.norm(B)
        assert abs(up @ bh - um @ bh) <= 2e-15 * max(nm, 1.0)
        pm = um - (um @ bh) * bh
        pp = up - (up @ bh) * bh
        angle = np.arctan2(np.cross(pm, pp) @ bh, pm @ pp)
        gm = np.sqrt(1.0 + um @ um)
        ref = -np.sign(qm) * 2.0 * np.arctan(abs(eps) * np.linalg.norm(B) / gm)
        # the angle is defined only as well as the perpendicular part is
        assert abs(angle - ref) <= 4e-15 * max(nm, 1.0) / max(np.linalg.norm(pm), 1e-300)


def test_boris_parallel_fields_accelerate_along_b(orc):
    """E parallel to B: the momentum along B gains (q/m) E dt exactly and the
    perpendicular part rotates by the Boris angle at gamma^-."""
    rng = np.random.default_rng(6)
    for _ in range(50):
        bh = rng.normal(size=3)
        bh /= np.linalg.norm(bh)
        Eamp, Bamp = rng.uniform(-2, 2), rng.uniform(0.1, 3)
        u = rng.normal(size=3) * 4
        qm, dt = float(rng.choice([-1.0, 1.0])), rng.uniform(0.1, 0.8)
        out = orc.boris(u, Eamp * bh, Bamp * bh, qm, dt)
        assert abs(out @ bh - (u @ bh + qm * Eamp * dt)) <= 1e-13 * max(1.0, abs(u @ bh))
        um = u + 0.5 * qm * dt * Eamp * bh
        gm = np.sqrt(1.0 + um @ um)
        pm = u - (u @ bh) * bh
        pp = out - (out @ bh) * bh
        angle = np.arctan2(np.cross(pm, pp) @ bh, pm @ pp)
        ref = -np.sign(qm) * 2.0 * np.arctan(0.5 * dt * Bamp / gm)
        assert abs(angle - ref) <= 1e-13


# ---------------------------------------------------------------------------
# Out-of-plane current in 2D
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("l", [1, 2, 3, 4])
def test_2d_out_of_plane_current_is_3d_path_summed_over_x3(orc, l):
    """In 3D the current along x3 of a path that advances dz = v_z dt / dx3
    cells, summed over the x3 nodes and times dx3, is Q v_z / (dx1 dx2) times
    the path average of S_x S_y (the x3 first moment of the B-spline moves by
    exactly dz).
    That is the 2D J3 of the same (x1, x2) path: the 2D weight of J3 must be
    the exact average along the straight path, which the 1/3 on DS_x DS_y
    expresses."""
    rng = np.random.default_rng(70 + l)
    n = (12, 11, 16)
    dxs = (1.0, 0.8, 1.3)
    dt = 0.35
    g3 = orc.Grid(3, n, l, dt, dx=dxs)
    g2 = orc.Grid(2, n[:2], l, dt, dx=dxs)
    for _ in range(20):
        x0 = np.array([rng.uniform(0, n[0]), rng.uniform(0, n[1]), rng.uniform(4, 12)])
        d = np.array([rng.uniform(-0.9, 0.9), rng.uniform(-0.9, 0.9), 0.0])
        vz = rng.uniform(-0.9, 0.9)
        Q = rng.uniform(0.5, 2.0)
        x1 = x0 + d
        x1[2] = x0[2] + vz * dt / dxs[2]
        g3.zero_J()
        g3.deposit(x0, x1, Q)
        summed = g3.J[2].reshape(n[2], n[1] * n[0]).sum(axis=0) * dxs[2]
        g2.zero_J()
        x0_2, x1_2 = x0.copy(), x1.copy()
        x0_2[2] = x1_2[2] = 0.0
        g2.deposit(x0_2, x1_2, Q, vz)
        scale = np.max(np.abs(g2.J[2]))
        # the x3 prefix sums cancel to a few 1e-14 of the scale
        assert np.max(np.abs(summed - g2.J[2])) <= 1e-12 * scale


# ---------------------------------------------------------------------------
# Energy sums of the Sec. 4 observable
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ndim", [2, 3])
def test_field_energy_of_cosine_modes(orc, ndim):
    """1/2 sum cos^2(2 pi m.x / N) A^2 Vc = 1/2 A^2 (ncell / 2) Vc for a mode
    that is neither constant nor at the Nyquist wavenumber; a constant
    component holds 1/2 A^2 ncell Vc."""
    n = (12, 10, 8)[:ndim]
    dxs = (1.0, 0.7, 1.3)
    g = orc.Grid(ndim, n, 2, 0.3, dx=dxs)
    Vc = float(np.prod(dxs[:ndim]))
    idx = np.arange(g.ncell)
    i = idx % g.n[0]
    j = (idx // g.n[0]) % g.n[1]
    k = idx // (g.n[0] * g.n[1])
    phase = 2 * np.pi * (3 * i / g.n[0] + 2 * j / g.n[1] + (1 * k / g.n[2] if ndim == 3 else 0.0))
    amps_E = (0.7, 1.9, 0.0)
    amps_B = (2.3, 0.0, 0.4)
    for d in range(3):
        g.E[d] = amps_E[d] * np.cos(phase + d)
        g.B[d] = amps_B[d] * np.sin(phase - d)
    g.E[2] = 0.25  # constant
    UE, UB = g.field_energy()
    ref_E = [0.5 * amps_E[0] ** 2 * g.ncell / 2 * Vc, 0.5 * amps_E[1] ** 2 * g.ncell / 2 * Vc,
             0.5 * 0.25 ** 2 * g.ncell * Vc]
    ref_B = [0.5 * a * a * g.ncell / 2 * Vc for a in amps_B]
    for d in range(3):
        assert abs(UE[d] - ref_E[d]) <= 1e-13 * max(ref_E[d], 1.0)
        assert abs(UB[d] - ref_B[d]) <= 1e-13 * max(ref_B[d], 1.0)


def test_kinetic_energy_integer_gamma(orc):
    """Momenta with |u|^2 = 0, 3, 8, 15, 24 have gamma = 1, 2, 3, 4, 5, so
    the kinetic energy is M c^2 (0 + 1 + 2 + 3 + 4) for any macro mass M and
    any c."""
    u = np.array([[0.0, 0.0, 0.0], [1.0, 1.0, 1.0], [2.0, 2.0, 0.0], [3.0, -1.0, np.sqrt(5.0)],
                  [2.0, -2.0, 4.0]])
    g = orc.Grid(2, (8, 8), 2, 0.3, c=1.7)
    for M in (1.0, 0.37, 250.0):
        assert abs(g.kinetic(u, M) - M * 1.7 ** 2 * 10.0) <= 1e-13 * M * 1.7 ** 2 * 10.0


# ---------------------------------------------------------------------------
# Fourth-order dispersion of M4 (Appendix C)
# ---------------------------------------------------------------------------

def _phase_error(orc, solver, a, n, m):
    """Relative phase-velocity error of the vacuum mode E3 = cos(k.x) on an
    n[0] x n[1] grid, k = 2 pi m / n.  The leapfrog advances every Fourier
    mode by a fixed rotation, so its projection p_s on cos(k.x) obeys
    p_{s+1} + p_{s-1} = 2 cos(theta) p_s; theta is fitted from the oracle's
    own steps and compared with the exact omega dt = c |k| dt."""
    g = orc.Grid(2, n, 2, a, solver=solver)
    i = np.arange(g.ncell) % n[0]
    j = np.arange(g.ncell) // n[0]
    k1, k2 = 2 * np.pi * m[0] / n[0], 2 * np.pi * m[1] / n[1]
    mode = np.cos(k1 * i + k2 * j)
    g.E[2] = mode
    p = [mode @ g.E[2]]
    for _ in range(12):
        g.field_update()
        p.append(mode @ g.E[2])
    p = np.array(p)
    lhs = p[2:] + p[:-2]
    rhs = 2.0 * p[1:-1]
    cos_theta = float(lhs @ rhs / (rhs @ rhs))
    theta = np.arccos(cos_theta)
    return theta / (a * np.hypot(k1, k2)) - 1.0


@pytest.mark.parametrize("m", [(1, 0), (1, 1), (2, 1)], ids=["along-x1", "diagonal", "oblique"])
def test_m4_dispersion_is_fourth_order(orc, m):
    """Halving |k| (same mode index on twice the grid) divides the phase
    error by ~16 with M4 and by ~4 with Yee."""
    a = 0.5
    ratios = {}
    for solver in (0, 1):
        e1 = _phase_error(orc, solver, a, (32, 32), m)
        e2 = _phase_error(orc, solver, a, (64, 64), m)
        ratios[solver] = e1 / e2
        assert e1 < 0 and e2 < 0   # both schemes are slower than light here
    assert 3.8 <= ratios[0] <= 4.2, ratios
    assert 15.0 <= ratios[1] <= 17.0, ratios


# ---------------------------------------------------------------------------
# Precision of the deposit for short transverse steps
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("l", [1, 2, 3, 4])
def test_transverse_current_of_tiny_steps(orc, ndim, l):
    """A beam particle moves ~1e-4 cells or less across the drift per step.
    Its transverse current still integrates to Q d / dt with the relative
    precision of FP64 arithmetic (sum J Vc = Q v, the continuity of Sec. 1),
    which needs S1 - S0 formed without cancelling the step against values of
    order one.  Steps down to 5e-6 cells, a tenth of the workloads' typical
    transverse step (extended precision keeps ~1e-18 absolute through the
    B-spline recurrence)."""
    rng = np.random.default_rng(90 + 10 * ndim + l)
    n = (10, 9, 8)
    g = orc.Grid(ndim, n[:ndim], l, 0.45)
    for step in (1e-4, 1e-5):
        for _ in range(5):
            x0 = np.array([rng.uniform(0, n[d]) if d < ndim else 0.0 for d in range(3)])
            d = np.array([rng.uniform(0.2, 0.45), step * rng.choice([-1, 1]) * rng.uniform(0.5, 1), 0.0])
            if ndim == 3:
                d[2] = step * rng.choice([-1, 1]) * rng.uniform(0.5, 1)
            Q = 1.0
            x1 = x0 + d
            g.zero_J()
            g.deposit(x0, x1, Q, 0.0)
            for k in range(1, ndim):
                # the step the particle takes: x1 - x0 is exact (Sterbenz)
                ref = Q * (x1[k] - x0[k]) / g.s.dt
                assert abs(g.J[k].sum() * g.Vc - ref) <= 1e-12 * abs(ref), (k, step)
