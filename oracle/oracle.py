"""ctypes wrapper around the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg.  The GPU library never imports or links it, and
it imports nothing from the GPU package.  See oracle.h for the conventions
(positions in cell units, u = gamma v / c, 4 pi absorbed in Maxwell).
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

WT, MC = 0, 1
YEE, M4 = 0, 1


def build():
    """Compile oracle.c into liboracle.so (plain gcc, no FMA contraction)."""
    cmd = [
        "gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
        os.path.join(HERE, "oracle.c"), "-o", LIB_PATH, "-lm",
    ]
    subprocess.run(cmd, check=True)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        _lib = ctypes.CDLL(LIB_PATH)
        _declare(_lib)
    return _lib


_dp = ctypes.POINTER(ctypes.c_double)


class OrcGrid(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("order", ctypes.c_int),
        ("scheme", ctypes.c_int), ("solver", ctypes.c_int), ("dx", ctypes.c_double * 3),
        ("dt", ctypes.c_double), ("c", ctypes.c_double),
        ("E", _dp * 3), ("B", _dp * 3), ("J", _dp * 3),
    ]


def _declare(L):
    d, i, l_ = ctypes.c_double, ctypes.c_int, ctypes.c_long
    g = ctypes.POINTER(OrcGrid)
    sig = {
        "orc_W": (d, [i, d]), "orc_C": (d, [i, d]), "orc_T": (d, [i, d, d]),
        "orc_W_vec": (None, [i, _dp, _dp, l_]), "orc_C_vec": (None, [i, _dp, _dp, l_]),
        "orc_T_vec": (None, [i, d, _dp, _dp, l_]),
        "orc_gather": (None, [g, _dp, _dp, _dp]),
        "orc_boris": (None, [_dp, _dp, _dp, d, d, d]),
        "orc_move": (None, [g, _dp, _dp]),
        "orc_deposit": (None, [g, _dp, _dp, d, d]),
        "orc_wrap": (None, [g, _dp]),
        "orc_zero_J": (None, [g]),
        "orc_push_species": (None, [g, l_, _dp, _dp, d, d]),
        "orc_perturbed": (i, [g, _dp, _dp, _dp, d]),
        "orc_push_species_skip": (None, [g, l_, _dp, _dp, d, d, _dp, _dp, d]),
        "orc_faraday_half": (None, [g]), "orc_ampere": (None, [g]),
        "orc_field_update": (None, [g]),
        "orc_rho": (None, [g, l_, _dp, d, _dp]),
        "orc_div_E": (None, [g, _dp]),
        "orc_field_energy": (None, [g, _dp, _dp]),
        "orc_kinetic": (d, [l_, _dp, d, d]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args


def _ptr(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


def _vec(fn, *args, y):
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.empty_like(y)
    fn(*args, _ptr(y), _ptr(out), y.size)
    return out


def W(l, y):
    """B-spline W_l evaluated elementwise."""
    return _vec(lib().orc_W_vec, l, y=y)


def C(l, z):
    """Integral of W_{l-1} from -inf to z, elementwise."""
    return _vec(lib().orc_C_vec, l, y=z)


def T(l, a, y):
    """WT factor T_l(y; a) elementwise."""
    return _vec(lib().orc_T_vec, l, float(a), y=y)


class Grid:
    """Fields and run constants of one periodic run, owned by numpy."""

    def __init__(self, ndim, n, order, dt, dx=(1.0, 1.0, 1.0), c=1.0, scheme=WT, solver=YEE):
        n = tuple(int(v) for v in n) + (1,) * (3 - len(n))
        if ndim == 2:
            n = (n[0], n[1], 1)
        self.ndim, self.n = ndim, n
        self.ncell = n[0] * n[1] * n[2]
        self.E = np.zeros((3, self.ncell))
        self.B = np.zeros((3, self.ncell))
        self.J = np.zeros((3, self.ncell))
        self.s = OrcGrid()
        self.s.ndim, self.s.order, self.s.scheme, self.s.solver = ndim, order, scheme, solver
        for d in range(3):
            self.s.n[d] = n[d]
            self.s.dx[d] = float(dx[d])
        self.s.dt, self.s.c = float(dt), float(c)
        self._bind()

    def _bind(self):
        for d in range(3):
            self.s.E[d] = self.E[d].ctypes.data_as(_dp)
            self.s.B[d] = self.B[d].ctypes.data_as(_dp)
            self.s.J[d] = self.J[d].ctypes.data_as(_dp)

    @property
    def ref(self):
        return ctypes.byref(self.s)

    @property
    def Vc(self):
        v = 1.0
        for d in range(self.ndim):
            v *= self.s.dx[d]
        return v

    def field_view(self, arr):
        """(3, n2, n1, n0) view of a field array (z, y, x order)."""
        return arr.reshape(3, self.n[2], self.n[1], self.n[0])

    # -- per-particle -----------------------------------------------------
    def gather(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(3)
        Ep, Bp = np.zeros(3), np.zeros(3)
        lib().orc_gather(self.ref, _ptr(x), _ptr(Ep), _ptr(Bp))
        return Ep, Bp

    def gather_many(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        E = np.zeros((len(x), 3))
        B = np.zeros((len(x), 3))
        for p in range(len(x)):
            E[p], B[p] = self.gather(x[p])
        return E, B

    def deposit(self, x0, x1, Q, vz=0.0):
        x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(3)
        x1 = np.ascontiguousarray(x1, dtype=np.float64).reshape(3)
        lib().orc_deposit(self.ref, _ptr(x0), _ptr(x1), float(Q), float(vz))

    # -- whole-run steps ----------------------------------------------------
    def zero_J(self):
        lib().orc_zero_J(self.ref)

    def push_species(self, x, u, qm, Q, skip=None):
        """Gather + Boris + move + deposit (+ wrap) for one species, in place.

        skip = (lo, hi, t): particles outside the region perturbed at time t
        around the box lo..hi only drift (partially skipped calculation)."""
        assert x.shape == u.shape and x.shape[1] == 3
        if skip is None:
            lib().orc_push_species(self.ref, len(x), _ptr(x), _ptr(u), float(qm), float(Q))
        else:
            lo, hi, t = skip
            lo = np.ascontiguousarray(lo, dtype=np.float64).reshape(3)
            hi = np.ascontiguousarray(hi, dtype=np.float64).reshape(3)
            lib().orc_push_species_skip(self.ref, len(x), _ptr(x), _ptr(u), float(qm), float(Q),
                                        _ptr(lo), _ptr(hi), float(t))

    def perturbed(self, x, lo, hi, t):
        """1 where the canonical positions x (np, 3) lie in the region
        perturbed at time t around the box lo..hi."""
        x = np.ascontiguousarray(x, dtype=np.float64).reshape(-1, 3)
        lo = np.ascontiguousarray(lo, dtype=np.float64).reshape(3)
        hi = np.ascontiguousarray(hi, dtype=np.float64).reshape(3)
        return np.array([lib().orc_perturbed(self.ref, _ptr(np.ascontiguousarray(x[p])), _ptr(lo), _ptr(hi),
                                             float(t)) for p in range(len(x))], dtype=np.int32)

    def field_update(self):
        lib().orc_field_update(self.ref)

    def faraday_half(self):
        lib().orc_faraday_half(self.ref)

    def ampere(self):
        lib().orc_ampere(self.ref)

    def step(self, species, skip=None):
        """One PIC step: zero J, push every species, update the fields.

        species: list of dicts with keys x, u (arrays (np, 3)), qm, Q;
        skip: as for push_species.
        """
        self.zero_J()
        for s in species:
            self.push_species(s["x"], s["u"], s["qm"], s["Q"], skip)
        self.field_update()

    # -- diagnostics --------------------------------------------------------
    def rho(self, species):
        out = np.zeros(self.ncell)
        for s in species:
            x = np.ascontiguousarray(s["x"], dtype=np.float64)
            lib().orc_rho(self.ref, len(x), _ptr(x), float(s["Q"]), _ptr(out))
        return out

    def div_E(self):
        out = np.zeros(self.ncell)
        lib().orc_div_E(self.ref, _ptr(out))
        return out

    def gauss_residual(self, species):
        return self.div_E() - self.rho(species)

    def field_energy(self):
        UE, UB = np.zeros(3), np.zeros(3)
        lib().orc_field_energy(self.ref, _ptr(UE), _ptr(UB))
        return UE, UB

    def kinetic(self, u, M):
        u = np.ascontiguousarray(u, dtype=np.float64)
        return lib().orc_kinetic(len(u), _ptr(u), float(M), float(self.s.c))


def boris(u, E, B, qm, dt, c=1.0):
    u = np.array(u, dtype=np.float64).reshape(3)
    E = np.ascontiguousarray(E, dtype=np.float64).reshape(3)
    B = np.ascontiguousarray(B, dtype=np.float64).reshape(3)
    lib().orc_boris(_ptr(u), _ptr(E), _ptr(B), float(qm), float(dt), float(c))
    return u
