"""The absolute-contribution scale of the mixed-precision current checks
(tests/helpers.abs_current_scale, built from two sign-split oracle deposits
per component) equals the brute-force sum over particles of the absolute
values of each particle's own current, node by node."""
import numpy as np
import pytest

from paper_1909_09613_amd.inputs import RunSpec
from tests import helpers as H


@pytest.mark.parametrize("spec", [
    RunSpec(2, (12, 10), 3, 0.45, 50.0, 0.01, 2, 5),
    RunSpec(2, (12, 10), 2, 0.6, 5.0, 0.3, 2, 6, colocated=False, drift_axis=1),
    RunSpec(3, (8, 8, 9), 2, 0.5, 20.0, 0.05, 1, 7),
], ids=["2d-beam", "2d-warm-drift-x2", "3d-beam"])
def test_abs_scale_is_sum_of_absolute_contributions(orc, spec):
    sp, E, B = H.random_state(spec, 3, 0.05)
    got = H.abs_current_scale(orc, spec, sp, E, B)
    g = H.oracle_grid(orc, spec)
    g.E[:] = E
    g.B[:] = B
    brute = np.zeros((3, spec.ncell))
    one = H.oracle_grid(orc, spec)
    for s in sp:
        x0 = s["x"].copy()
        x1 = s["x"].copy()
        u = s["u"].copy()
        g.push_species(x1, u, s["qm"], s["Q"])
        for p in range(len(x0)):
            d = H.min_image(x1[p] - x0[p], np.array(spec.n3, dtype=float))
            d[spec.ndim:] = 0.0
            gam = np.sqrt(1.0 + u[p] @ u[p])
            one.zero_J()
            one.deposit(x0[p], x0[p] + d, s["Q"], spec.c * u[p, 2] / gam)
            brute += np.abs(one.J)
    ref = brute.max(axis=1)
    assert np.all(np.abs(got - ref) <= 1e-12 * ref)
