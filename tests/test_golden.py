"""The shock-tube generators reproduce the initial states printed in section 5.1
(fixture: tests/golden/shock_tube_states.txt)."""
import os

import numpy as np

from paper_1102_5202_amd import workloads as WL

HERE = os.path.dirname(os.path.abspath(__file__))


def load_states():
    out = {}
    with open(os.path.join(HERE, "golden", "shock_tube_states.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t, side, *vals = line.split()
            out[(t, side)] = np.array([float(v) for v in vals])
    return out


def test_shock_tube_states_match_paper():
    st = load_states()
    for name, mag in (("sod", False), ("balsara1", True)):
        w = WL.sod(n=10, magnetised=mag)
        assert w.gamma == 5.0 / 3.0
        for side, cell in (("L", 0), ("R", 9)):
            ref = st[(name, side)]
            P = w.P[:, 0, 0, cell]
            np.testing.assert_array_equal(P[[0, 1]], ref[[0, 1]])
            np.testing.assert_array_equal(P[2:5], ref[2:5])     # W = 1: u~ = v = 0
            np.testing.assert_array_equal(P[5:8], ref[5:8])
            assert P[8] == 0.0
