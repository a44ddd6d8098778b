"""Seeded synthetic inputs: the drifting pair plasma both the GPU path and the
CPU oracle consume.

This module only draws and arranges numbers; it contains none of the PIC
step's arithmetic, and it serves the tests and the benchmark, which hand the
same arrays to both sides.

Recipe (the paper's test problem, Table 1, with the sizes of the workload
being run):
  * exactly ``ppc_s`` particles per cell per species, uniform within the cell
    (stratified), positrons co-located with electrons unless ``colocated`` is
    False, so rho = 0 and E = B = 0 satisfy Gauss's law at t = 0;
  * co-moving momenta u' ~ N(0, u_th^2) per component via Box-Muller
    (Appendix D names Box-Muller for the Maxwell-Boltzmann limit);
  * the volume-transform correction of Appendix D as a flip of u'_x: keep u'
    with probability (1 + beta v'_x)/2, otherwise reflect it.  This is the
    reading under which the reflected sample carries the Jacobian
    (1 + beta v'_x); the inequality as printed selects the opposite branch;
  * Lorentz boost along +x1: u_x = gamma0 (u'_x + beta0 gamma'), u_perp = u'_perp
    (or along another axis, ``drift_axis``, with the components relabelled);
  * macro charge |Q| = gamma0 Vc omega_pe^2 / ppc_s with omega_pe = c / d_e and
    d_e = ``skin_depth_cells`` cells (Table 1: 256 cells = 16 d_e), macro mass
    M = |Q|, q/m = -1 (electrons) and +1 (positrons).
"""
from dataclasses import dataclass, field

import numpy as np


@dataclass
class RunSpec:
    ndim: int
    n: tuple                      # cells per axis (2 or 3 entries)
    order: int                    # B-spline order l
    courant: float                # c dt / dx (dx = 1, c = 1)
    gamma0: float = 50.0
    u_th: float = 0.01
    ppc_s: int = 4                # particles per cell per species
    seed: int = 1001
    scheme: int = 0               # 0 = WT, 1 = MC
    solver: int = 0               # 0 = Yee, 1 = M4
    skin_depth_cells: float = 16.0
    colocated: bool = True
    dx: tuple = field(default=(1.0, 1.0, 1.0))
    c: float = 1.0
    drift_axis: int = 0           # axis of the drift (0 = x1, the paper's beam direction)

    @property
    def ncell(self):
        return int(np.prod(self.n))

    @property
    def dt(self):
        return self.courant * self.dx[0] / self.c

    @property
    def n3(self):
        return tuple(self.n) + (1,) * (3 - len(self.n))

    @property
    def Vc(self):
        return float(np.prod(self.dx[: self.ndim]))

    def species_constants(self):
        """[(q/m, Q, M)] for electrons and positrons."""
        wpe = self.c / (self.skin_depth_cells * self.dx[0])
        q = self.gamma0 * self.Vc * wpe * wpe / self.ppc_s
        return [(-1.0, -q, q), (1.0, q, q)]


def box_muller(rng, n):
    """n standard normals from uniform pairs (Box & Muller 1958)."""
    m = (n + 1) // 2
    u1 = 1.0 - rng.random(m)          # (0, 1]
    u2 = rng.random(m)
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.concatenate([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)])
    return z[:n]


def drifting_momenta(rng, n, gamma0, u_th, axis=0):
    """(n, 3) momenta u = gamma v / c of a plasma drifting along +x_axis
    (axis 0 is x1).  The draws do not depend on the axis: the components are
    drawn as for a drift along x1 and then relabelled."""
    up = box_muller(rng, 3 * n).reshape(3, n).T * u_th
    gp = np.sqrt(1.0 + np.sum(up * up, axis=1))
    beta0 = np.sqrt(1.0 - 1.0 / (gamma0 * gamma0))
    vpx = up[:, 0] / gp
    x1 = rng.random(n)
    flip = (1.0 + beta0 * vpx) / 2.0 < x1
    up[flip, 0] = -up[flip, 0]
    u = up.copy()
    u[:, 0] = gamma0 * (up[:, 0] + beta0 * gp)
    if axis != 0:
        u[:, [0, axis]] = u[:, [axis, 0]]
    return u


def stratified_positions(rng, spec, p0, p1):
    """(p1 - p0, 3) positions in cell units of particles p0..p1-1, where
    particle p sits in cell p // ppc_s (cell-major, x fastest)."""
    n3 = spec.n3
    cell = np.arange(p0, p1, dtype=np.int64) // spec.ppc_s
    base = np.empty((p1 - p0, 3), dtype=np.float64)
    base[:, 0] = cell % n3[0]
    base[:, 1] = (cell // n3[0]) % n3[1]
    base[:, 2] = cell // (n3[0] * n3[1])
    off = rng.random((p1 - p0, 3))
    if spec.ndim == 2:
        off[:, 2] = 0.0
    x = base + off
    # an offset that rounds the position onto the upper cell face stays in range
    for d in range(spec.ndim):
        x[:, d] = np.where(x[:, d] >= n3[d], 0.0, x[:, d])
    return x


CHUNK = 1 << 20   # particles per independent random stream


def make_species(spec, workers=None):
    """Electron and positron arrays for one run.

    Particles are drawn in chunks of about CHUNK particles (whole cells), each
    from its own PCG64 stream spawned from ``spec.seed``, so that large
    workloads are generated in parallel and the result does not depend on
    the number of workers.  Returns a list of dicts {x, u, qm, Q, M} with x, u
    of shape (np, 3).
    """
    from concurrent.futures import ThreadPoolExecutor
    import os

    n = spec.ncell * spec.ppc_s
    per = max(1, CHUNK // spec.ppc_s) * spec.ppc_s
    bounds = [(p, min(p + per, n)) for p in range(0, n, per)]
    seeds = np.random.SeedSequence(spec.seed).spawn(len(bounds))
    xe = np.empty((n, 3))
    xp = xe if spec.colocated else np.empty((n, 3))
    ue = np.empty((n, 3))
    up = np.empty((n, 3))

    def fill(k):
        p0, p1 = bounds[k]
        rng = np.random.Generator(np.random.PCG64(seeds[k]))
        xe[p0:p1] = stratified_positions(rng, spec, p0, p1)
        if not spec.colocated:
            xp[p0:p1] = stratified_positions(rng, spec, p0, p1)
        ue[p0:p1] = drifting_momenta(rng, p1 - p0, spec.gamma0, spec.u_th, spec.drift_axis)
        up[p0:p1] = drifting_momenta(rng, p1 - p0, spec.gamma0, spec.u_th, spec.drift_axis)

    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    if len(bounds) == 1 or workers <= 1:
        for k in range(len(bounds)):
            fill(k)
    else:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(fill, range(len(bounds))))
    if spec.colocated:
        xp = xe.copy()
    out = []
    for (qm, Q, M), x, u in zip(spec.species_constants(), (xe, xp), (ue, up)):
        out.append({"x": x, "u": u, "qm": qm, "Q": Q, "M": M})
    return out


def quantize_fp32(x, u):
    """Round a state onto the FP32 layout (int32 cell + FP32 offset, FP32 u),
    returned as float64 arrays holding exactly representable values."""
    cell = np.floor(x)
    off = (x - cell).astype(np.float32).astype(np.float64)
    carry = off >= 1.0
    off[carry] = 0.0
    cell[carry] += 1.0
    return cell + off, u.astype(np.float32).astype(np.float64)


def random_fields(rng, ncell, amp):
    """(3, ncell) uniform random field components in [-amp, amp)."""
    return (2.0 * rng.random((3, ncell)) - 1.0) * amp


def config(k):
    """The five benchmark workloads as RunSpec lists (k = 1..5).

    1: 2D 64x64, l=2, C=0.7, gamma 50, 4 ppc/species, FP64 correctness case.
    2: 2D 1024x512, l=3, C=0.45, gamma 50, 16 ppc/species.
    3: 3D 256x128x128, l=2, C=0.5, gamma 50, 8 ppc/species.
    4: 64 runs, 2D grids U{128..512} x U{64..256}, l=2, C_r = 0.1 + 0.6 r/63,
       gamma in (10, 50, 100), 8 ppc/species.
    5: 2D 4096x2048, l=3, C=0.3, gamma 100, 16 ppc/species.
    """
    if k == 1:
        return [RunSpec(2, (64, 64), 2, 0.7, 50.0, 0.01, 4, 1001)]
    if k == 2:
        return [RunSpec(2, (1024, 512), 3, 0.45, 50.0, 0.01, 16, 1002)]
    if k == 3:
        return [RunSpec(3, (256, 128, 128), 2, 0.5, 50.0, 0.01, 8, 1003)]
    if k == 4:
        rng = np.random.Generator(np.random.PCG64(4000))
        runs = []
        for r in range(64):
            n1 = int(rng.integers(128, 513))
            n2 = int(rng.integers(64, 257))
            cr = (10.0 + 60.0 * r / 63.0) / 100.0
            if r == 42:
                cr = 0.5
            runs.append(RunSpec(2, (n1, n2), 2, cr, (10.0, 50.0, 100.0)[r % 3], 0.01, 8, 4001 + r))
        return runs
    if k == 5:
        return [RunSpec(2, (4096, 2048), 3, 0.3, 100.0, 0.01, 16, 1005)]
    raise ValueError(k)
