"""Pins of the oracle's gather, Boris push, deposit, Maxwell solvers and whole
step against what the paper and the mathematics fix: the component-by-
component structure of Eq. interpolation-EB-real-mod (with the printed T_l),
exactness on uniform and linear fields, the MC limit, Boris closed forms,
discrete continuity (Sec. 1, exact charge conservation), the Yee and M4
dispersion relations (Appendix C), conservation of Gauss's law (Appendix B),
the electrostatic self-force statements that hold on the staggered grid
(Appendix B), and the cold-plasma oscillation frequency."""
import numpy as np
import pytest

from tests.paper_printed import PRINTED_T


def _grid(orc, ndim=2, n=(12, 10, 1), l=2, a=0.3, scheme=0, solver=0):
    return orc.Grid(ndim, n[:ndim] if ndim == 3 else n[:2], l, a, scheme=scheme, solver=solver)


# ---------------------------------------------------------------------------
# Gather
# ---------------------------------------------------------------------------

# (component, staggered axes) for E1..E3, B1..B3 on the Yee grid (Sec. 2)
STAGGER = {
    ("E", 0): (0.5, 0.0), ("E", 1): (0.0, 0.5), ("E", 2): (0.0, 0.0),
    ("B", 0): (0.0, 0.5), ("B", 1): (0.5, 0.0), ("B", 2): (0.5, 0.5),
}
# WT kernel per axis in 2D (x1, x2), Eq. interpolation-EB-real-mod
WT_KIND = {
    ("E", 0): ("W", "T"), ("E", 1): ("T", "W"), ("E", 2): ("T", "T"),
    ("B", 0): ("T", "W"), ("B", 1): ("W", "T"), ("B", 2): ("W", "W"),
}


@pytest.mark.parametrize("l", [1, 2, 3, 4])
@pytest.mark.parametrize("a", [0.15, 0.45])
def test_gather_single_node_matches_equation(orc, l, a):
    """A field that is 1 on one node and 0 elsewhere gathers to the product
    of the kernels the interpolation equation names for that component,
    evaluated at the node's staggered position.  T from the printed
    polynomials, W from the oracle's B-spline (pinned separately)."""
    rng = np.random.default_rng(11 * l)
    g = _grid(orc, n=(16, 16, 1), l=l, a=a)
    kern = {"W": lambda y: orc.W(l, np.array([y]))[0], "T": lambda y: PRINTED_T[l](np.array([y]), a)[0]}
    for (fld, comp), lam in STAGGER.items():
        for _ in range(6):
            node = (int(rng.integers(4, 12)), int(rng.integers(4, 12)))
            x = np.array([node[0] + rng.uniform(-2, 2), node[1] + rng.uniform(-2, 2), 0.0])
            g.E[:] = 0
            g.B[:] = 0
            arr = g.E if fld == "E" else g.B
            arr[comp][node[0] + 16 * node[1]] = 1.0
            Ep, Bp = g.gather(x)
            got = (Ep if fld == "E" else Bp)[comp]
            k1, k2 = WT_KIND[(fld, comp)]
            ref = kern[k1](x[0] - node[0] - lam[0]) * kern[k2](x[1] - node[1] - lam[1])
            assert abs(got - ref) <= 1e-13
            other = Bp if fld == "E" else Ep
            assert np.all(other == 0)


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("l", [1, 2, 3, 4])
@pytest.mark.parametrize("scheme", [0, 1])
def test_gather_uniform_and_linear_fields(orc, ndim, l, scheme):
    """Uniform fields are gathered exactly for every l (partition of unity);
    fields linear along an axis are reproduced exactly for l >= 2."""
    n = (24, 20, 16)
    g = orc.Grid(ndim, n[:ndim], l, 0.37, scheme=scheme)
    rng = np.random.default_rng(3)
    cE, cB = rng.normal(size=3), rng.normal(size=3)
    g.E[:] = cE[:, None]
    g.B[:] = cB[:, None]
    for _ in range(10):
        x = np.array([rng.uniform(8, 14), rng.uniform(8, 12), rng.uniform(6, 10) if ndim == 3 else 0.0])
        Ep, Bp = g.gather(x)
        assert np.allclose(Ep, cE, rtol=0, atol=1e-14)
        assert np.allclose(Bp, cB, rtol=0, atol=1e-14)
    if l < 2:
        return
    # linear in x2 (no wrap inside the sampled region): f = alpha + beta * x2
    n3 = g.n
    jj = (np.arange(g.ncell) // n3[0]) % n3[1]
    for (fld, comp), lam in STAGGER.items():
        arr = g.E if fld == "E" else g.B
        arr[:] = 0
        arr[comp] = 0.7 + 0.3 * (jj + lam[1])
        for _ in range(5):
            x = np.array([rng.uniform(8, 14), rng.uniform(7, 12), rng.uniform(6, 10) if ndim == 3 else 0.0])
            Ep, Bp = g.gather(x)
            got = (Ep if fld == "E" else Bp)[comp]
            assert abs(got - (0.7 + 0.3 * x[1])) <= 1e-13


@pytest.mark.parametrize("l", [1, 2, 3, 4])
def test_wt_equals_mc_at_half_courant(orc, l):
    """For c dt = dx/2 the WT tensor equals the MC tensor (Sec. 2)."""
    rng = np.random.default_rng(l)
    gw = orc.Grid(2, (16, 12), l, 0.5, scheme=orc.WT)
    gm = orc.Grid(2, (16, 12), l, 0.5, scheme=orc.MC)
    for g in (gw, gm):
        g.E[:] = rng.normal(size=g.E.shape) if g is gw else gw.E
        g.B[:] = rng.normal(size=g.B.shape) if g is gw else gw.B
    for _ in range(20):
        x = np.array([rng.uniform(0, 16), rng.uniform(0, 12), 0.0])
        e1, b1 = gw.gather(x)
        e2, b2 = gm.gather(x)
        assert np.max(np.abs(e1 - e2)) <= 1e-14 and np.max(np.abs(b1 - b2)) <= 1e-14


# ---------------------------------------------------------------------------
# Boris
# ---------------------------------------------------------------------------

def test_boris_uniform_E(orc):
    rng = np.random.default_rng(1)
    for _ in range(20):
        u = rng.normal(size=3) * 10
        E = rng.normal(size=3)
        qm, dt = rng.choice([-1.0, 1.0]), rng.uniform(0.05, 0.9)
        out = orc.boris(u, E, np.zeros(3), qm, dt)
        assert np.allclose(out, u + qm * E * dt, rtol=0, atol=1e-13)


def test_boris_uniform_B_rotation(orc):
    """With E = 0 the push is a rotation about B by -2 atan(|t|) (sign of q),
    t = (q/m) B dt / (2 gamma); |u| is conserved."""
    rng = np.random.default_rng(2)
    for _ in range(20):
        u = rng.normal(size=3) * 5
        B = rng.normal(size=3)
        qm, dt = rng.choice([-1.0, 1.0]), rng.uniform(0.05, 0.9)
        gam = np.sqrt(1 + u @ u)
        t = qm * B * dt / (2 * gam)
        theta = -2 * np.arctan(np.linalg.norm(t)) * np.sign(qm)
        bh = B / np.linalg.norm(B)
        # Rodrigues rotation of u about bh by theta
        ref = u * np.cos(theta) + np.cross(bh, u) * np.sin(theta) + bh * (bh @ u) * (1 - np.cos(theta))
        out = orc.boris(u, np.zeros(3), B, qm, dt)
        assert np.allclose(out, ref, rtol=0, atol=1e-12)
        assert abs(np.linalg.norm(out) - np.linalg.norm(u)) <= 1e-12


# ---------------------------------------------------------------------------
# Deposit
# ---------------------------------------------------------------------------

def _continuity_residual(orc, g, x0, x1, Q):
    """(rho1 - rho0)/dt + D.J for one particle, D the Gauss operator."""
    g.zero_J()
    g.deposit(x0, x1, Q, vz=0.123)
    sp0 = [{"x": x0.reshape(1, 3), "Q": Q}]
    x1w = x1.copy().reshape(1, 3)
    for d in range(g.ndim):
        x1w[0, d] %= g.n[d]
    sp1 = [{"x": x1w, "Q": Q}]
    rho0, rho1 = g.rho(sp0), g.rho(sp1)
    saveE = g.E.copy()
    g.E[:] = g.J
    divJ = g.div_E()
    g.E[:] = saveE
    return (rho1 - rho0) / g.s.dt + divJ, rho0


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("l", [1, 2, 3, 4])
def test_deposit_discrete_continuity(orc, ndim, l):
    rng = np.random.default_rng(10 * ndim + l)
    n = (10, 9, 8)
    g = orc.Grid(ndim, n[:ndim], l, 0.6)
    for _ in range(25):
        x0 = np.array([rng.uniform(0, n[d]) if d < ndim else 0.0 for d in range(3)])
        dx = np.array([rng.uniform(-0.95, 0.95) if d < ndim else 0.0 for d in range(3)])
        # include tiny transverse steps, as in a beam drifting along x1
        if rng.random() < 0.5:
            dx[1] *= 1e-4
        Q = rng.uniform(0.5, 2.0)
        res, rho0 = _continuity_residual(orc, g, x0, x0 + dx, Q)
        assert np.max(np.abs(res)) <= 1e-13 * Q / g.s.dt


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("l", [1, 3])
def test_deposit_discrete_continuity_anisotropic_cells(orc, ndim, l):
    """Continuity with cells of different size along each axis (the current
    scales -Q dx_d/(Vc dt) and the divergence 1/dx_d must match)."""
    rng = np.random.default_rng(40 + 10 * ndim + l)
    n = (10, 9, 8)
    g = orc.Grid(ndim, n[:ndim], l, 0.3, dx=(1.0, 0.7, 1.3))
    for _ in range(15):
        x0 = np.array([rng.uniform(0, n[d]) if d < ndim else 0.0 for d in range(3)])
        dx = np.array([rng.uniform(-0.95, 0.95) if d < ndim else 0.0 for d in range(3)])
        Q = rng.uniform(0.5, 2.0)
        res, rho0 = _continuity_residual(orc, g, x0, x0 + dx, Q)
        assert np.max(np.abs(res)) <= 1e-13 * Q / (g.s.dt * 0.7 * (1.3 if ndim == 3 else 1.0))


@pytest.mark.parametrize("ndim", [2, 3])
@pytest.mark.parametrize("l", [1, 2, 3, 4])
def test_deposit_total_current(orc, ndim, l):
    """sum_cells J Vc = Q v: the current of one particle integrates to its
    charge times its velocity (J3 in 2D: Q vz)."""
    rng = np.random.default_rng(20 + ndim + l)
    n = (10, 9, 8)
    g = orc.Grid(ndim, n[:ndim], l, 0.6)
    for _ in range(10):
        x0 = np.array([rng.uniform(0, n[d]) if d < ndim else 0.0 for d in range(3)])
        dx = np.array([rng.uniform(-0.95, 0.95) if d < ndim else 0.0 for d in range(3)])
        Q, vz = 1.3, 0.4
        g.zero_J()
        g.deposit(x0, x0 + dx, Q, vz)
        for d in range(ndim):
            assert abs(g.J[d].sum() * g.Vc - Q * dx[d] / g.s.dt) <= 1e-13
        if ndim == 2:
            assert abs(g.J[2].sum() * g.Vc - Q * vz) <= 1e-13


@pytest.mark.parametrize("l", [1, 2, 3, 4])
def test_deposit_1d_reduction(orc, l):
    """A particle moving only along x1 carries across the face f = m1 + 1/2
    the charge that W_l puts on nodes right of f, sum_{n > f} W_l(x - n),
    which equals the integral of W_{l-1}(s - f) over s < x.  Hence
    J1(f, m2) dt = Q W_l(x2 - m2) * integral of W_{l-1}(s - f) over [x0, x1].
    Integral by Gauss-Legendre on the oracle's W (pinned to s_l)."""
    rng = np.random.default_rng(30 + l)
    g = orc.Grid(2, (14, 12), l, 0.6)
    xg, wg = np.polynomial.legendre.leggauss(30)
    for _ in range(6):
        x0 = np.array([rng.uniform(4, 8), rng.uniform(4, 8), 0.0])
        x1 = x0 + np.array([rng.uniform(-0.9, 0.9), 0.0, 0.0])
        Q = 0.9
        g.zero_J()
        g.deposit(x0, x1, Q)
        J1 = g.J[0].reshape(12, 14)
        for m1 in range(14):
            f = m1 + 0.5
            knots = np.arange(-l / 2, l / 2 + 0.5) + f
            lo, hi = min(x0[0], x1[0]), max(x0[0], x1[0])
            pts = np.concatenate([[lo], knots[(knots > lo) & (knots < hi)], [hi]])
            integ = 0.0
            for p, q in zip(pts[:-1], pts[1:]):
                s = 0.5 * (q - p) * xg + 0.5 * (q + p)
                integ += np.sum(wg * 0.5 * (q - p) * orc.W(l - 1, s - f))
            integ *= np.sign(x1[0] - x0[0])
            for m2 in range(12):
                ref = Q * integ / g.s.dt * orc.W(l, np.array([x0[1] - m2]))[0]
                assert abs(J1[m2, m1] - ref) <= 1e-14
        assert np.all(g.J[1] == 0.0)


# ---------------------------------------------------------------------------
# Maxwell solvers
# ---------------------------------------------------------------------------

def _mode_theta(solver, a, ks, dxs=(1.0, 1.0, 1.0)):
    """sin^2(theta/2) = (c dt)^2 sum_i s_i^2 A_i, s_i = sin(k_i dx_i/2)/dx_i
    (Appendix C; A_i = 1 for Yee)."""
    cdt = a * dxs[0]
    tot = 0.0
    for i, k in enumerate(ks):
        s = np.sin(k * dxs[i] / 2) / dxs[i]
        A = 1.0
        if solver == 1:
            for j, kj in enumerate(ks):
                c2 = (cdt / dxs[j]) ** 2
                coef = (c2 - 1) / 12 if j == i else c2 / 12
                A -= 2 * coef * (1 - np.cos(kj * dxs[j]))
        tot += s * s * A
    return 2 * np.arcsin(cdt * np.sqrt(tot))


@pytest.mark.parametrize("solver", [0, 1])
@pytest.mark.parametrize("a", [0.2, 0.5, 0.7])
def test_vacuum_mode_dispersion_2d(orc, solver, a):
    n = (16, 12)
    m1, m2 = 3, 2
    k1, k2 = 2 * np.pi * m1 / n[0], 2 * np.pi * m2 / n[1]
    g = orc.Grid(2, n, 2, a, solver=solver)
    i = np.arange(g.ncell) % n[0]
    j = np.arange(g.ncell) // n[0]
    E30 = np.cos(k1 * i + k2 * j)
    g.E[2] = E30
    th = _mode_theta(solver, a, (k1, k2))
    for step in range(1, 41):
        g.field_update()
        assert np.max(np.abs(g.E[2] - np.cos(step * th) * E30)) <= 1e-12
    assert np.max(np.abs(g.E[:2])) <= 1e-12


@pytest.mark.parametrize("solver", [0, 1])
def test_vacuum_mode_dispersion_2d_anisotropic_cells(orc, solver):
    """A vacuum mode on cells of 1 x 0.7 advances by the phase of the
    dispersion relation with per-axis dx (Appendix C, A_i with per-axis
    coefficients)."""
    n = (16, 12)
    dxs = (1.0, 0.7, 1.0)
    a = 0.45
    m1, m2 = 3, 2
    k1, k2 = 2 * np.pi * m1 / (n[0] * dxs[0]), 2 * np.pi * m2 / (n[1] * dxs[1])
    g = orc.Grid(2, n, 2, a * dxs[0], dx=dxs, solver=solver)
    i = np.arange(g.ncell) % n[0]
    j = np.arange(g.ncell) // n[0]
    E30 = np.cos(2 * np.pi * m1 * i / n[0] + 2 * np.pi * m2 * j / n[1])
    g.E[2] = E30
    th = _mode_theta(solver, a, (k1, k2), dxs)
    for step in range(1, 31):
        g.field_update()
        assert np.max(np.abs(g.E[2] - np.cos(step * th) * E30)) <= 1e-12


@pytest.mark.parametrize("solver", [0, 1])
def test_vacuum_mode_dispersion_3d(orc, solver):
    n = (6, 10, 8)
    a = 0.45
    k2, k3 = 2 * np.pi * 3 / n[1], 2 * np.pi * 1 / n[2]
    g = orc.Grid(3, n, 2, a, solver=solver)
    j = (np.arange(g.ncell) // n[0]) % n[1]
    k = np.arange(g.ncell) // (n[0] * n[1])
    E10 = np.cos(k2 * j + k3 * k)
    g.E[0] = E10
    th = _mode_theta(solver, a, (0.0, k2, k3))
    for step in range(1, 31):
        g.field_update()
        assert np.max(np.abs(g.E[0] - np.cos(step * th) * E10)) <= 1e-12


@pytest.mark.parametrize("ndim", [2, 3])
def test_ampere_keeps_divergence(orc, ndim):
    """D.(curl B) = 0: with J = 0 the Gauss residual does not change."""
    n = (8, 7, 6)
    g = orc.Grid(ndim, n[:ndim], 2, 0.4, solver=1)
    rng = np.random.default_rng(4)
    g.B[:] = rng.normal(size=g.B.shape)
    g.E[:] = rng.normal(size=g.E.shape)
    d0 = g.div_E()
    for _ in range(5):
        g.field_update()
    assert np.max(np.abs(g.div_E() - d0)) <= 1e-12


# ---------------------------------------------------------------------------
# Whole step
# ---------------------------------------------------------------------------

def _species(spec):
    from paper_1909_09613_amd import inputs

    return inputs.make_species(spec)


def test_gauss_law_preserved(orc):
    """Appendix B: with a charge-conserving deposit D.E - rho keeps its
    initial value (here nonzero: independent electron/positron positions)."""
    from paper_1909_09613_amd.inputs import RunSpec

    spec = RunSpec(2, (16, 12), 2, 0.7, 50.0, 0.05, 2, 77, colocated=False, skin_depth_cells=3.0)
    sp = _species(spec)
    g = orc.Grid(2, spec.n, spec.order, spec.dt)
    r0 = g.gauss_residual(sp)
    assert np.max(np.abs(r0)) > 1e-3
    for _ in range(20):
        g.step(sp)
    r = g.gauss_residual(sp)
    assert np.max(np.abs(g.E)) > 1e-4
    assert np.max(np.abs(r - r0)) <= 1e-12


@pytest.mark.parametrize("l", [2, 4])
def test_wt_step_equals_mc_step_at_half_courant(orc, l):
    from paper_1909_09613_amd.inputs import RunSpec

    spec = RunSpec(2, (12, 10), l, 0.5, 20.0, 0.05, 2, 5, colocated=False, skin_depth_cells=3.0)
    sw, sm = _species(spec), _species(spec)
    gw = orc.Grid(2, spec.n, l, spec.dt, scheme=orc.WT)
    gm = orc.Grid(2, spec.n, l, spec.dt, scheme=orc.MC)
    for _ in range(6):
        gw.step(sw)
        gm.step(sm)
    for a, b in zip(sw, sm):
        assert np.max(np.abs(a["x"] - b["x"])) <= 1e-13
        assert np.max(np.abs(a["u"] - b["u"])) <= 1e-12
    assert np.max(np.abs(gw.E - gm.E)) <= 1e-14 * max(1.0, np.max(np.abs(gw.E)))


@pytest.mark.parametrize("scheme", [0, 1])
def test_cold_pair_plasma_oscillation(orc, scheme):
    """A cold pair plasma with a small velocity perturbation oscillates at
    omega^2 = omega_e^2 + omega_p^2 = 2 omega_pe^2 (long-wavelength limit);
    the leapfrog, the finite particle shape and k = 2 pi/32 shift it by well
    under 2 %.  Exercises gather, push, move, deposit and Ampere together."""
    from paper_1909_09613_amd.inputs import RunSpec

    spec = RunSpec(2, (32, 4), 2, 0.3, 1.0, 0.0, 8, 9, skin_depth_cells=4.0, scheme=scheme)
    sp = _species(spec)
    L = spec.n[0]
    eps = 1e-3
    sp[0]["u"][:, :] = 0.0
    sp[1]["u"][:, :] = 0.0
    sp[0]["u"][:, 0] = eps * np.sin(2 * np.pi * sp[0]["x"][:, 0] / L)
    g = orc.Grid(2, spec.n, spec.order, spec.dt, scheme=scheme)
    series = []
    nsteps = 240
    for _ in range(nsteps):
        g.step(sp)
        series.append(g.E[0][5])
    s = np.array(series)
    t = (np.arange(nsteps) + 1) * spec.dt
    zc = [t[i] - s[i] * (t[i + 1] - t[i]) / (s[i + 1] - s[i]) for i in range(nsteps - 1) if s[i] * s[i + 1] < 0]
    period = 2 * np.mean(np.diff(zc))
    omega = 2 * np.pi / period
    wpe = 1.0 / spec.skin_depth_cells
    assert abs(omega / (np.sqrt(2) * wpe) - 1) < 0.02


# ---------------------------------------------------------------------------
# Electrostatic self-force (Appendix B)
# ---------------------------------------------------------------------------

def _self_field(orc, g, x, Q=1.0):
    """Periodic electrostatic field of one particle on the Yee lattice:
    -Lap5 phi = rho (neutralising background), E_d = -(phi(m+e_d) - phi(m))/dx."""
    rho = g.rho([{"x": x.reshape(1, 3), "Q": Q}]).reshape(g.n[1], g.n[0])
    k0 = 2 * np.pi * np.fft.fftfreq(g.n[0])
    k1 = 2 * np.pi * np.fft.fftfreq(g.n[1])
    K2 = (2 * np.sin(k1[:, None] / 2)) ** 2 + (2 * np.sin(k0[None, :] / 2)) ** 2
    rk = np.fft.fft2(rho)
    K2[0, 0] = 1.0
    phik = rk / K2
    phik[0, 0] = 0.0
    phi = np.real(np.fft.ifft2(phik))
    return phi


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("l", [1, 2, 3, 4])
def test_self_force_staggered_symmetry(orc, scheme, l):
    """On the staggered grid F_self,1 vanishes where x1 is a multiple of 1/2
    and is odd about those points (reflection maps both lattices onto
    themselves); its cell average is therefore zero."""
    n = (16, 16)
    g = orc.Grid(2, n, l, 0.3, scheme=scheme)
    rng = np.random.default_rng(40 + l)
    for _ in range(4):
        p = 6 + 0.5 * int(rng.integers(0, 4))
        x2 = rng.uniform(5, 11)
        forces = {}
        for dlt in (0.0, 0.13, -0.13):
            x = np.array([p + dlt, x2, 0.0])
            phi = _self_field(orc, g, x)
            E1 = -(np.roll(phi, -1, axis=1) - phi)
            E2 = -(np.roll(phi, -1, axis=0) - phi)
            g.E[:] = 0
            g.B[:] = 0
            g.E[0] = E1.ravel()
            g.E[1] = E2.ravel()
            Ep, _ = g.gather(x)
            forces[dlt] = Ep[0]
        assert abs(forces[0.0]) <= 1e-15
        assert abs(forces[0.13] + forces[-0.13]) <= 1e-15
        assert abs(forces[0.13]) > 1e-6


@pytest.mark.parametrize("scheme", [0, 1])
@pytest.mark.parametrize("l", [2, 3, 4])
def test_self_force_vanishes_collocated(orc, scheme, l):
    """Appendix B's argument where its assumption holds: with E_1 on the rho
    lattice (centred difference, antisymmetric Green's function) and the WT
    (or MC) weights W_l(x1) T_l(x2), F_self,1 = 0 at any position."""
    n = (16, 16)
    a = 0.3
    g = orc.Grid(2, n, l, a)
    rng = np.random.default_rng(50 + l)
    for _ in range(6):
        x = np.array([rng.uniform(4, 12), rng.uniform(4, 12), 0.0])
        phi = _self_field(orc, g, x)
        E1c = -(np.roll(phi, -1, axis=1) - np.roll(phi, 1, axis=1)) / 2
        m1 = np.arange(n[0])
        m2 = np.arange(n[1])
        w1 = orc.W(l, x[0] - m1)
        w2 = orc.T(l, a, x[1] - m2) if scheme == 0 else orc.W(l, x[1] - m2)
        F1 = np.sum(E1c * w2[:, None] * w1[None, :])
        assert abs(F1) <= 1e-16
