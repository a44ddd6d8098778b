"""Pins of the oracle's partially skipped calculation (Sec. 3, "Partially
skipping calculation"): the perturbed region A(t) is the set of points closer
than c t to the initially perturbed region A0, and outside it the particles
only drift (momentum kept, no current).

  * membership against the set definition itself, by brute force over a
    dense sample of A0 and its periodic images, with anisotropic cells;
  * A(0) = A0, and on-axis distances across the periodic boundary;
  * a skipped particle keeps u bit for bit and moves by (c dt/dx) u/gamma,
    the closed form of pure drift, and adds no current;
  * a particle inside takes exactly the full step, and a box covering the
    whole domain reproduces the plain step bit for bit.
"""
import numpy as np
import pytest

N = (12, 10)
DX = (1.0, 0.7)


def _grid(orc, n=N, dx=DX, l=2, dt=0.3):
    return orc.Grid(2, n, l, dt, dx=(dx[0], dx[1], 1.0))


def _brute_distance(x, lo, hi, n, dx, h=0.05):
    """Euclidean distance (physical units) from each x to a lattice of
    spacing <= h over the box lo..hi (edges included) and its eight
    periodic neighbours, and the lattice's covering radius."""
    ax = [np.linspace(lo[d], hi[d], max(2, int(np.ceil((hi[d] - lo[d]) / h)) + 1)) for d in range(2)]
    gx, gy = np.meshgrid(ax[0], ax[1], indexing="ij")
    pts = []
    for kx in (-1, 0, 1):
        for ky in (-1, 0, 1):
            pts.append(np.stack([(gx + kx * n[0]).ravel(), (gy + ky * n[1]).ravel()], axis=1))
    pts = np.concatenate(pts)
    step = [(hi[d] - lo[d]) / (len(ax[d]) - 1) if len(ax[d]) > 1 else 0.0 for d in range(2)]
    cover = 0.5 * np.hypot(step[0] * dx[0], step[1] * dx[1])
    out = np.empty(len(x))
    for p in range(len(x)):
        dd = (pts - x[p, :2]) * np.array(dx)
        out[p] = np.sqrt(np.min(np.sum(dd * dd, axis=1)))
    return out, cover


@pytest.mark.parametrize("box", [((3.2, 4.1), (5.5, 6.0)), ((0.0, 7.5), (1.5, 10.0)), ((10.5, 0.2), (12.0, 2.0))])
@pytest.mark.parametrize("ct", [0.0, 0.9, 2.6, 4.3])
def test_membership_matches_set_definition(orc, box, ct):
    """x is in A(t) when some point of A0 (or of a periodic image) lies
    closer than c t; at t = 0, A(0) = A0."""
    g = _grid(orc)
    lo = np.array([box[0][0], box[0][1], 0.0])
    hi = np.array([box[1][0], box[1][1], 0.0])
    rng = np.random.default_rng(11)
    x = np.zeros((400, 3))
    x[:, 0] = rng.random(400) * N[0]
    x[:, 1] = rng.random(400) * N[1]
    got = g.perturbed(x, lo, hi, ct)  # c = 1
    dist, cover = _brute_distance(x, lo, hi, N, DX)
    inside = np.all((x[:, :2] >= lo[:2]) & (x[:, :2] <= hi[:2]), axis=1)
    if ct == 0.0:
        assert np.array_equal(got.astype(bool), inside)
        return
    clear = np.abs(dist - ct) > cover + 1e-12
    assert clear.sum() > 300
    assert np.array_equal(got[clear].astype(bool), dist[clear] < ct)
    assert np.all(got[inside] == 1)


def test_membership_on_axis_and_across_the_periodic_boundary(orc):
    g = _grid(orc)
    lo = np.array([1.0, 2.0, 0.0])
    hi = np.array([2.0, 3.0, 0.0])
    # 1.5 cells to the right of the box along x (physical 1.5 * dx0)
    x = np.array([[3.5, 2.5, 0.0]])
    assert g.perturbed(x, lo, hi, 1.49)[0] == 0
    assert g.perturbed(x, lo, hi, 1.51)[0] == 1
    # through the periodic end: from x = n - 0.75 = 11.25 the nearest image
    # of [1, 2] is [13, 14], 1.75 cells away
    x = np.array([[N[0] - 0.75, 2.5, 0.0]])
    assert g.perturbed(x, lo, hi, 1.74)[0] == 0
    assert g.perturbed(x, lo, hi, 1.76)[0] == 1
    # along y the cells are 0.7 wide: 2 cells above the box is 1.4
    x = np.array([[1.5, 5.0, 0.0]])
    assert g.perturbed(x, lo, hi, 1.39)[0] == 0
    assert g.perturbed(x, lo, hi, 1.41)[0] == 1
    # diagonal: 3 cells right and 2 cells up from the corner (2, 3)
    x = np.array([[5.0, 5.0, 0.0]])
    r = np.hypot(3.0, 1.4)
    assert g.perturbed(x, lo, hi, r - 1e-9)[0] == 0
    assert g.perturbed(x, lo, hi, r + 1e-9)[0] == 1


def _state(orc, n_per=300, seed=5):
    g = _grid(orc, l=3, dt=0.4)
    rng = np.random.default_rng(seed)
    for d in range(3):
        g.E[d] = 0.05 * rng.standard_normal(g.ncell)
        g.B[d] = 0.05 * rng.standard_normal(g.ncell)
    x = np.zeros((n_per, 3))
    x[:, 0] = rng.random(n_per) * N[0]
    x[:, 1] = rng.random(n_per) * N[1]
    u = rng.standard_normal((n_per, 3)) * np.array([3.0, 0.5, 0.5])
    return g, x, u


def test_skipped_particles_drift_and_deposit_nothing(orc):
    g, x, u = _state(orc)
    lo, hi, t = np.array([4.0, 3.0, 0.0]), np.array([6.0, 5.0, 0.0]), 1.7
    inside = g.perturbed(x, lo, hi, t).astype(bool)
    assert 30 < inside.sum() < len(x) - 30
    xs, us = x.copy(), u.copy()
    g.zero_J()
    g.push_species(xs, us, -1.0, -0.01, skip=(lo, hi, t))
    J_skip = g.J.copy()
    # outside: pure drift, closed form
    out = ~inside
    assert np.array_equal(us[out], u[out])
    gam = np.sqrt(1.0 + np.sum(u[out] ** 2, axis=1))
    for d in range(2):
        xd = x[out, d] + (g.s.c * g.s.dt / DX[d]) * (u[out, d] / gam)
        xd = np.mod(xd, N[d])
        assert np.max(np.abs(xs[out, d] - xd)) <= 1e-13
    # inside: the full step, and all of the current
    xi, ui = x[inside].copy(), u[inside].copy()
    g.zero_J()
    g.push_species(xi, ui, -1.0, -0.01)
    assert np.array_equal(xs[inside], xi) and np.array_equal(us[inside], ui)
    assert np.array_equal(J_skip, g.J)


def test_box_covering_the_domain_is_the_plain_step(orc):
    g, x, u = _state(orc, seed=6)
    xa, ua = x.copy(), u.copy()
    g.zero_J()
    g.push_species(xa, ua, 1.0, 0.02, skip=(np.zeros(3), np.array([N[0], N[1], 0.0]), 0.0))
    Ja = g.J.copy()
    xb, ub = x.copy(), u.copy()
    g.zero_J()
    g.push_species(xb, ub, 1.0, 0.02)
    assert np.array_equal(xa, xb) and np.array_equal(ua, ub) and np.array_equal(Ja, g.J)


def test_nothing_perturbed_means_no_current(orc):
    """t = 0 and A0 away from every particle: the whole species drifts."""
    g, x, u = _state(orc, seed=7)
    keep = ~((x[:, 0] >= 5.0) & (x[:, 0] <= 5.5) & (x[:, 1] >= 5.0) & (x[:, 1] <= 5.5))
    x, u = x[keep].copy(), u[keep].copy()
    u0 = u.copy()
    g.zero_J()
    g.push_species(x, u, -1.0, -0.01, skip=(np.array([5.0, 5.0, 0.0]), np.array([5.5, 5.5, 0.0]), 0.0))
    assert np.array_equal(u, u0)
    assert not np.any(g.J)
