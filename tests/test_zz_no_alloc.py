"""pic_init_static, the allocation-free initialisation (its scratch is a
device array of the library), through the C-ABI: a context it creates steps
to the same state as a context of pic_init with caller-owned scratch, on two
calls in a row (each destroyed before the next), the second with a smaller
problem, so that whatever the first left in the shared array must not leak
into the second.  Also: a second live context on the device is refused, and
so is a problem whose scratch exceeds the array.

Bounds are those of the parity tests (both sides are the same kernels, so
they differ only by the order of the FP64 current atomics): FP64 positions
1e-12 cells, momenta and fields 1e-12 relative; mixed precision 2e-6.
"""
import ctypes

import numpy as np
import pytest

import paper_1909_09613_amd as wt
from paper_1909_09613_amd import inputs
from paper_1909_09613_amd.inputs import RunSpec
from tests import helpers as H

pytestmark = pytest.mark.gpu

STEPS = 11   # one captured graph of 8 steps and three eager steps


class StaticSim:
    """A context of pic_init_static with torch-owned particle, field and
    current buffers and no scratch buffer."""

    def __init__(self, spec, precision):
        import torch

        self.spec = spec
        self.descs = [wt.make_desc(spec, precision)]
        need = wt.pic_query_layout(self.descs)
        self.device = torch.device("cuda:0")
        self.buffers = [torch.empty(max(b, 256), dtype=torch.uint8, device=self.device) for b in need[:3]]
        self.stream = torch.cuda.Stream(device=self.device)
        torch.cuda.synchronize(self.device)
        b = wt.pic_buffers()
        b.particles, b.fields, b.current = [t.data_ptr() for t in self.buffers]
        b.scratch = None
        for k in range(3):
            b.bytes[k] = self.buffers[k].numel()
        b.bytes[3] = 0
        self.ctx = wt.pic_init_static(self.descs, b, self.stream.cuda_stream)

    def close(self):
        if self.ctx is not None:
            wt.pic_destroy(self.ctx)
            self.ctx = None


def _run(sim, spec, sp, E, B):
    ctx = sim.ctx
    for s in range(2):
        wt.pic_set_particles(ctx, 0, s, sp[s]["x"], sp[s]["u"])
    wt.pic_set_fields(ctx, 0, E, B)
    wt.pic_step(ctx, STEPS)
    d = wt.pic_diagnostics(ctx, 0)
    assert d.n_nonfinite == 0 and d.n_out_of_range == 0
    got = [wt.pic_get_particles(ctx, 0, s, spec.ncell * spec.ppc_s) for s in range(2)]
    Eg, Bg, _ = wt.pic_get_fields(ctx, 0, spec.ncell)
    return got, Eg, Bg, d


CALLS = [
    (RunSpec(2, (96, 64), 3, 0.45, 50.0, 0.01, 4, 301), wt.PIC_FP64),
    (RunSpec(2, (48, 40), 2, 0.6, 20.0, 0.05, 3, 302, colocated=False), wt.PIC_MIXED32),
]


def test_static_scratch_matches_caller_scratch_twice():
    for spec, precision in CALLS:
        fp32 = precision == wt.PIC_MIXED32
        sp, E, B = H.random_state(spec, 5, 0.05, fp32=fp32)
        ref = wt.Sim([spec], precision)
        try:
            want, Ew, Bw, dw = _run(ref, spec, sp, E, B)
        finally:
            ref.close()
        st = StaticSim(spec, precision)
        try:
            got, Eg, Bg, dg = _run(st, spec, sp, E, B)
        finally:
            st.close()
        tol = 2e-6 if fp32 else 1e-12
        wanted = [{"x": x, "u": u} for x, u in want]
        ex, eu = H.particle_errors(spec, wanted, got)
        eE = max(H.rel_maxnorm(Eg, Ew))
        eB = max(H.rel_maxnorm(Bg, Bw))
        print("static scratch %s %s: dx=%.2e du=%.2e dE=%.2e dB=%.2e" % (
            "x".join(map(str, spec.n)), "fp32" if fp32 else "fp64", ex, eu, eE, eB), flush=True)
        assert ex <= tol and eu <= tol
        assert eE <= (1e-5 if fp32 else 1e-12) and eB <= (1e-5 if fp32 else 1e-12)
        assert dg.step == dw.step == STEPS


def test_static_scratch_one_context_per_device_and_size_limit():
    spec = RunSpec(2, (40, 32), 2, 0.45, 50.0, 0.01, 2, 303)
    first = StaticSim(spec, wt.PIC_FP64)
    try:
        with pytest.raises(wt.PicError) as ei:
            StaticSim(spec, wt.PIC_FP64)
        assert ei.value.status == wt.PIC_ERR_STATE
    finally:
        first.close()
    again = StaticSim(spec, wt.PIC_FP64)   # released by pic_destroy
    again.close()
    big = RunSpec(2, (1024, 512), 3, 0.45, 50.0, 0.01, 16, 304)
    with pytest.raises(wt.PicError) as ei:
        StaticSim(big, wt.PIC_MIXED32)
    assert ei.value.status == wt.PIC_ERR_ARG
    assert "static scratch" in wt.pic_last_error()
