"""Writes printed_T.txt: values of the paper's printed T_1..T_4 (Sec. 2, the
piecewise equations after Eq. tau_l, 0 < c dt/dx <= 1/2) on a small grid of
(y, a).  Columns: l, a, y, T_l(y; a).  Run from the repository root:
    python tests/golden/make_printed_T.py
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from tests.paper_printed import PRINTED_T  # noqa: E402

rows = []
for l in (1, 2, 3, 4):
    for a in (0.05, 0.2, 0.35, 0.5):
        for y in np.linspace(-(l / 2 + a) - 0.25, l / 2 + a + 0.25, 13):
            rows.append((l, a, y, float(PRINTED_T[l](np.array([y]), a)[0])))
out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "printed_T.txt")
with open(out, "w") as f:
    f.write("# l a y T_l(y;a) -- the paper's printed T_1..T_4 (Sec. 2), 48 dt~ read for 48 dt in T_4\n")
    for r in rows:
        f.write("%d %.17g %.17g %.17g\n" % r)
