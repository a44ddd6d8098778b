"""2D trajectories on the GPU against the FP64 oracle over graph-replayed
steps (pic_step), in both precisions, across the orders and stencil shapes
the one-step tests reach only once: linear to quartic B-splines, T_l with
l + 2 nodes (c dt > dx / 2), the MC scheme and the M4 Faraday stencil.
Carried from step to step: the tiles' boxes and windows, the fixed-point
bounds of the previous step, the re-sort, the field update between pushes.

Bounds as for the 3D trajectories: FP64 positions 1e-12 cells, momenta
1e-12 relative, E and B 1e-12 relative max-norm; mixed precision rounds to
FP32 every step, so 1e-4 in positions and momenta and 1e-3 in the fields.
"""
import pytest

import paper_1909_09613_amd as wt
from paper_1909_09613_amd.inputs import RunSpec
from tests import helpers as H

pytestmark = pytest.mark.gpu

CASES = {
    "linear": RunSpec(2, (40, 28), 1, 0.3, 50.0, 0.01, 3, 301),
    "cubic": RunSpec(2, (37, 29), 3, 0.45, 50.0, 0.01, 3, 302),
    "quartic": RunSpec(2, (36, 20), 4, 0.25, 20.0, 0.05, 2, 303),
    "a-above-half": RunSpec(2, (30, 26), 3, 0.6, 10.0, 0.1, 2, 304),
    "mc-scheme": RunSpec(2, (32, 32), 2, 0.3, 50.0, 0.01, 3, 305, scheme=1),
    "m4-solver": RunSpec(2, (34, 24), 2, 0.45, 50.0, 0.01, 3, 306, solver=1),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", [wt.PIC_FP64, wt.PIC_MIXED32], ids=["fp64", "fp32"])
def test_2d_multistep_against_oracle(orc, case, precision):
    ex, eu, eE, eB, _ = H.trajectory_vs_oracle(orc, CASES[case], 0.01, 16, precision)
    if precision == wt.PIC_FP64:
        assert ex <= 1e-12 and eu <= 1e-12
        assert eE <= 1e-12 and eB <= 1e-12
    else:
        assert ex <= 1e-4 and eu <= 1e-4
        assert eE <= 1e-3 and eB <= 1e-3
