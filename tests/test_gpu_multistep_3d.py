"""3D trajectories on the GPU against the FP64 oracle over many
graph-replayed steps (pic_step), in both precisions.  One-step tests cannot
reach the parts of the 3D particle kernel that carry state from one step to
the next:

  * a drifting beam (gamma 50 along x1 at c dt = 0.5 dx) moves its tiles'
    boxes half a cell per step, 16 cells (one period of the grid) in 32
    steps, with no re-sort: the staged windows follow the boxes across the
    periodic end;
  * a cold plasma at rest under strong random fields accelerates in every
    direction: in the first steps every particle's step exceeds twice the
    bound its tile recorded (the thermal velocities of the load), so its
    current takes the per-group coarse windows in global memory, which the
    flush reads and clears for the group's next tile; the plasma then spreads
    out of its tiles and is re-sorted (the count of sorts is checked);
  * the beam along x3 instead (drift_axis 2).

Bounds: FP64 positions 1e-12 cells, momenta 1e-12 relative, E and B 1e-12
relative max-norm.  Mixed precision starts from an FP32-representable state
and rounds to FP32 every step (~2e-6 per step, the one-step bound); over 20-32
steps that accumulates to at most ~1e-4 in positions and momenta, and the
fields, which sum the currents of all steps, to 1e-3 relative max-norm.
"""
import pytest

import paper_1909_09613_amd as wt
from paper_1909_09613_amd.inputs import RunSpec
from tests import helpers as H

pytestmark = pytest.mark.gpu

CASES = {
    "drifting-beam": (RunSpec(3, (16, 12, 10), 2, 0.5, 50.0, 0.01, 2, 201), 0.002, 32),
    "cold-start-strong-fields": (RunSpec(3, (14, 12, 10), 2, 0.45, 1.0, 0.001, 2, 202, colocated=False,
                                         skin_depth_cells=4.0), 0.3, 24),
    "beam-along-x3": (RunSpec(3, (12, 12, 18), 2, 0.5, 50.0, 0.01, 2, 203, drift_axis=2), 0.002, 24),
    # the 256-thread kernel of the higher orders, and l + 2 T nodes
    "cubic": (RunSpec(3, (12, 12, 12), 3, 0.35, 50.0, 0.01, 1, 204), 0.002, 20),
    "a-above-half": (RunSpec(3, (12, 10, 10), 2, 0.55, 10.0, 0.1, 2, 205), 0.002, 20),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", [wt.PIC_FP64, wt.PIC_MIXED32], ids=["fp64", "fp32"])
def test_3d_multistep_against_oracle(orc, case, precision):
    spec, amp, steps = CASES[case]
    ex, eu, eE, eB, sorts = H.trajectory_vs_oracle(orc, spec, amp, steps, precision)
    if precision == wt.PIC_FP64:
        assert ex <= 1e-12 and eu <= 1e-12
        assert eE <= 1e-12 and eB <= 1e-12
    else:
        assert ex <= 1e-4 and eu <= 1e-4
        assert eE <= 1e-3 and eB <= 1e-3
    if case == "cold-start-strong-fields":
        assert sorts >= 2   # the spreading plasma was re-sorted during the run
