"""MI355X-native hot path of a relativistic EM-PIC step with the WT force
interpolation of arXiv:1909.09613 (Lu, Kilian, Guo, Li, Liang).

This module is a thin ctypes binding of ``libwtpic.so`` (include/wtpic.h):
argument marshalling only.  Every step of the path runs in the library's HIP
kernels; PyTorch supplies device memory and the stream.  There is no CPU
fallback: importing works without the library, but any call that needs it
raises if ``libwtpic.so`` has not been built (``python -m
paper_1909_09613_amd.build``).
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwtpic.so")

PIC_OK, PIC_ERR_ARG, PIC_ERR_CFL, PIC_ERR_UNSUPPORTED = 0, -1, -2, -3
PIC_ERR_HIP, PIC_ERR_NUMERIC, PIC_ERR_STATE = -4, -5, -6
PIC_WT, PIC_MC = 0, 1
PIC_YEE, PIC_M4 = 0, 1
PIC_FP64, PIC_MIXED32 = 0, 1

STATUS_NAMES = {
    0: "PIC_OK", -1: "PIC_ERR_ARG", -2: "PIC_ERR_CFL", -3: "PIC_ERR_UNSUPPORTED",
    -4: "PIC_ERR_HIP", -5: "PIC_ERR_NUMERIC", -6: "PIC_ERR_STATE",
}

EXPORTED = [
    "pic_query_layout", "pic_init", "pic_init_static", "pic_set_particles", "pic_get_particles", "pic_set_fields",
    "pic_get_fields", "pic_gather_push_deposit", "pic_field_update", "pic_step", "pic_step_diag",
    "pic_diagnostics",
    "pic_set_tiling", "pic_autotune", "pic_tiling_candidates", "pic_set_skip_region", "pic_kernel_timing",
    "pic_last_error", "pic_destroy", "pic_table_weights",
]


class pic_run_desc(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("dx", ctypes.c_double * 3),
        ("c", ctypes.c_double), ("courant", ctypes.c_double), ("order", ctypes.c_int32),
        ("scheme", ctypes.c_int32), ("solver", ctypes.c_int32), ("drift_axis", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("ppc_per_species", ctypes.c_int32), ("q_over_m", ctypes.c_double * 2),
        ("macro_charge", ctypes.c_double * 2),
    ]


class pic_buffers(ctypes.Structure):
    _fields_ = [
        ("particles", ctypes.c_void_p), ("fields", ctypes.c_void_p), ("current", ctypes.c_void_p),
        ("scratch", ctypes.c_void_p), ("bytes", ctypes.c_size_t * 4),
    ]


class pic_diag(ctypes.Structure):
    _fields_ = [
        ("step", ctypes.c_int64), ("time", ctypes.c_double), ("UE", ctypes.c_double * 3),
        ("UB", ctypes.c_double * 3), ("Ekin", ctypes.c_double * 2), ("momentum", ctypes.c_double * 3),
        ("gauss_resid_max", ctypes.c_double), ("n_nonfinite", ctypes.c_int64),
        ("n_out_of_range", ctypes.c_int64), ("n_sorts", ctypes.c_int64),
    ]

    def as_dict(self):
        return {
            "step": self.step, "time": self.time, "UE": list(self.UE), "UB": list(self.UB),
            "Ekin": list(self.Ekin), "momentum": list(self.momentum),
            "gauss_resid_max": self.gauss_resid_max, "n_nonfinite": self.n_nonfinite,
            "n_out_of_range": self.n_out_of_range, "n_sorts": self.n_sorts,
        }


class PicError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


_lib = None


def lib():
    """The loaded libwtpic.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libwtpic.so is not built; run `python -m paper_1909_09613_amd.build` (no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        rd = ctypes.POINTER(pic_run_desc)
        sig = {
            "pic_query_layout": [rd, i32, ctypes.POINTER(ctypes.c_size_t)],
            "pic_init": [rd, i32, ctypes.POINTER(pic_buffers), vp, ctypes.POINTER(vp)],
            "pic_init_static": [rd, i32, ctypes.POINTER(pic_buffers), vp, ctypes.POINTER(vp)],
            "pic_set_particles": [vp, i32, i32, dp, dp, i64],
            "pic_get_particles": [vp, i32, i32, dp, dp, i64],
            "pic_set_fields": [vp, i32, dp, dp],
            "pic_get_fields": [vp, i32, dp, dp, dp],
            "pic_gather_push_deposit": [vp],
            "pic_field_update": [vp],
            "pic_step": [vp, i32],
            "pic_step_diag": [vp, i32, i32, i32, ctypes.POINTER(pic_diag)],
            "pic_diagnostics": [vp, i32, ctypes.POINTER(pic_diag)],
            "pic_set_tiling": [vp, ctypes.POINTER(i32), i32, i32],
            "pic_set_skip_region": [vp, i32, dp, dp, ctypes.c_double],
            "pic_kernel_timing": [vp, i32, dp, ctypes.POINTER(i64)],
            "pic_autotune": [vp, i32, ctypes.POINTER(i32), dp],
            "pic_tiling_candidates": [i32, i32, ctypes.POINTER(i32), i32, ctypes.POINTER(i32)],
            "pic_destroy": [vp],
            "pic_table_weights": [i32, i32, ctypes.c_double, ctypes.c_double, ctypes.POINTER(i32),
                                  ctypes.POINTER(i32), dp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.pic_last_error.argtypes = [vp]
        L.pic_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status, ctx=None):
    if status != PIC_OK:
        msg = lib().pic_last_error(ctx).decode(errors="replace")
        raise PicError(status, msg)


def _dptr(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_desc(spec, precision=PIC_MIXED32):
    """pic_run_desc from a RunSpec (paper_1909_09613_amd.inputs)."""
    d = pic_run_desc()
    d.ndim = spec.ndim
    n3 = spec.n3
    for k in range(3):
        d.n[k] = n3[k]
        d.dx[k] = spec.dx[k]
    d.c = spec.c
    d.courant = spec.courant
    d.order = spec.order
    d.scheme = spec.scheme
    d.solver = spec.solver
    d.drift_axis = spec.drift_axis
    d.precision = precision
    d.ppc_per_species = spec.ppc_s
    for s, (qm, Q, _M) in enumerate(spec.species_constants()):
        d.q_over_m[s] = qm
        d.macro_charge[s] = Q
    return d


# ---- C-ABI mirrors (same names as include/wtpic.h) --------------------------

def pic_query_layout(descs):
    arr = (pic_run_desc * len(descs))(*descs)
    out = (ctypes.c_size_t * 4)()
    _check(lib().pic_query_layout(arr, len(descs), out))
    return list(out)


def pic_init(descs, bufs, stream_handle):
    arr = (pic_run_desc * len(descs))(*descs)
    ctx = ctypes.c_void_p()
    _check(lib().pic_init(arr, len(descs), ctypes.byref(bufs), ctypes.c_void_p(stream_handle), ctypes.byref(ctx)))
    return ctx


def pic_init_static(descs, bufs, stream_handle):
    """pic_init with the library's static device scratch (bufs.scratch is
    ignored)."""
    arr = (pic_run_desc * len(descs))(*descs)
    ctx = ctypes.c_void_p()
    _check(lib().pic_init_static(arr, len(descs), ctypes.byref(bufs), ctypes.c_void_p(stream_handle),
                                 ctypes.byref(ctx)))
    return ctx


def pic_set_particles(ctx, run, species, x, u):
    x = np.ascontiguousarray(x, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    _check(lib().pic_set_particles(ctx, run, species, _dptr(x), _dptr(u), len(x)), ctx)


def pic_get_particles(ctx, run, species, n):
    x = np.zeros((n, 3))
    u = np.zeros((n, 3))
    _check(lib().pic_get_particles(ctx, run, species, _dptr(x), _dptr(u), n), ctx)
    return x, u


def pic_set_fields(ctx, run, E=None, B=None):
    Ec = None if E is None else np.ascontiguousarray(E, dtype=np.float64)
    Bc = None if B is None else np.ascontiguousarray(B, dtype=np.float64)
    _check(lib().pic_set_fields(ctx, run, None if Ec is None else _dptr(Ec), None if Bc is None else _dptr(Bc)), ctx)


def pic_get_fields(ctx, run, ncell):
    E, B, J = np.zeros((3, ncell)), np.zeros((3, ncell)), np.zeros((3, ncell))
    _check(lib().pic_get_fields(ctx, run, _dptr(E), _dptr(B), _dptr(J)), ctx)
    return E, B, J


def pic_gather_push_deposit(ctx):
    _check(lib().pic_gather_push_deposit(ctx), ctx)


def pic_field_update(ctx):
    _check(lib().pic_field_update(ctx), ctx)


def pic_step(ctx, n_steps):
    _check(lib().pic_step(ctx, n_steps), ctx)


def pic_step_diag(ctx, n_steps, diag_every, run):
    """n_steps steps; the diagnostics of `run` every diag_every steps."""
    n = n_steps // diag_every if diag_every > 0 else 0
    hist = (pic_diag * max(n, 1))()
    _check(lib().pic_step_diag(ctx, n_steps, diag_every, run, hist), ctx)
    return [hist[i] for i in range(n)]


def pic_diagnostics(ctx, run, allow_numeric=False):
    d = pic_diag()
    st = lib().pic_diagnostics(ctx, run, ctypes.byref(d))
    if not (allow_numeric and st == PIC_ERR_NUMERIC):
        _check(st, ctx)
    return d


def pic_set_tiling(ctx, tile=(0, 0, 0), margin=0, sort_every=0):
    t = (ctypes.c_int32 * 3)(*tile)
    _check(lib().pic_set_tiling(ctx, t, margin, sort_every), ctx)


def pic_set_skip_region(ctx, run, lo=None, hi=None, t0=0.0):
    """Partially skipped calculation for one run: the box lo..hi (cell
    units) is the initially perturbed region, t0 the time of the next step;
    lo=None switches it off."""
    if lo is None:
        _check(lib().pic_set_skip_region(ctx, run, None, None, 0.0), ctx)
        return
    def pad3(v):
        out = np.zeros(3)
        v = np.asarray(v, dtype=np.float64).ravel()
        out[:len(v)] = v
        return out

    lo, hi = pad3(lo), pad3(hi)
    _check(lib().pic_set_skip_region(ctx, run, lo.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     hi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(t0)), ctx)


def pic_kernel_timing(ctx, enable):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().pic_kernel_timing(ctx, 1 if enable else 0, ctypes.byref(ms), ctypes.byref(n)), ctx)
    return ms.value, n.value


def pic_autotune(ctx, trial_steps=16):
    """Times the candidate tilings on the context's own workload, applies the
    fastest and undoes the trial steps; returns the choice."""
    ch = (ctypes.c_int32 * 5)()
    ms = ctypes.c_double()
    _check(lib().pic_autotune(ctx, trial_steps, ch, ctypes.byref(ms)), ctx)
    return {"tile": tuple(ch[0:3]), "margin": ch[3], "sort_every": ch[4], "ms_per_step": ms.value}


def pic_tiling_candidates(ndim, precision):
    """The autotuner's candidate tilings, in trial order (the first is the
    default): list of dicts tile, margin, sort_every."""
    n = ctypes.c_int32()
    _check(lib().pic_tiling_candidates(ndim, precision, None, 0, ctypes.byref(n)))
    buf = (ctypes.c_int32 * (5 * max(n.value, 1)))()
    _check(lib().pic_tiling_candidates(ndim, precision, buf, n.value, ctypes.byref(n)))
    return [{"tile": tuple(buf[5 * i:5 * i + 3]), "margin": buf[5 * i + 3], "sort_every": buf[5 * i + 4]}
            for i in range(n.value)]


def pic_last_error(ctx=None):
    return lib().pic_last_error(ctx).decode(errors="replace")


def pic_destroy(ctx):
    _check(lib().pic_destroy(ctx))


def pic_table_weights(l, kind, a, f):
    first = ctypes.c_int32()
    cnt = ctypes.c_int32()
    w = np.zeros(8)
    _check(lib().pic_table_weights(l, kind, float(a), float(f), ctypes.byref(first), ctypes.byref(cnt), _dptr(w)))
    return first.value, w[: cnt.value].copy()


# ---- convenience: a context with torch-owned buffers --------------------------

class Sim:
    """Runs of one context, with device buffers owned by torch tensors.

    specs: RunSpec list (paper_1909_09613_amd.inputs); precision PIC_FP64 or
    PIC_MIXED32.  The context works on its own torch stream (`self.stream`).
    """

    def __init__(self, specs, precision=PIC_MIXED32, device="cuda:0"):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the WT PIC path runs only in its HIP kernels")
        lib()
        self.specs = list(specs)
        self.precision = precision
        self.descs = [make_desc(s, precision) for s in self.specs]
        self.bytes = pic_query_layout(self.descs)
        self.device = torch.device(device)
        self.buffers = [torch.empty(max(b, 256), dtype=torch.uint8, device=self.device) for b in self.bytes]
        self.stream = torch.cuda.Stream(device=self.device)
        torch.cuda.synchronize(self.device)
        b = pic_buffers()
        b.particles, b.fields, b.current, b.scratch = [t.data_ptr() for t in self.buffers]
        for k in range(4):
            b.bytes[k] = self.buffers[k].numel()
        self.ctx = pic_init(self.descs, b, self.stream.cuda_stream)

    def set_species(self, run, species_list):
        for s, sp in enumerate(species_list):
            pic_set_particles(self.ctx, run, s, sp["x"], sp["u"])

    def particles(self, run, species):
        spec = self.specs[run]
        return pic_get_particles(self.ctx, run, species, spec.ncell * spec.ppc_s)

    def fields(self, run):
        return pic_get_fields(self.ctx, run, self.specs[run].ncell)

    def set_fields(self, run, E=None, B=None):
        pic_set_fields(self.ctx, run, E, B)

    def gpd(self):
        pic_gather_push_deposit(self.ctx)

    def field_update(self):
        pic_field_update(self.ctx)

    def step(self, n=1):
        pic_step(self.ctx, n)

    def autotune(self, trial_steps=16):
        return pic_autotune(self.ctx, trial_steps)

    def set_skip_region(self, run, lo=None, hi=None, t0=0.0):
        pic_set_skip_region(self.ctx, run, lo, hi, t0)

    def step_diag(self, n, every, run=0):
        return pic_step_diag(self.ctx, n, every, run)

    def diagnostics(self, run=0, allow_numeric=False):
        return pic_diagnostics(self.ctx, run, allow_numeric)

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if self.ctx is not None:
            pic_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
