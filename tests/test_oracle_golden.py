"""Regression of the FP64 oracle against its committed fixture (see tests/golden/README.md)."""
import json
import os

import numpy as np

from oracle import dlr_oracle as O
from synth import problems

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_slab_beam_fixture():
    with open(os.path.join(HERE, "slab_beam_32_r8.json")) as f:
        ref = json.load(f)
    _, hist = O.run_dlr(problems.slab_beam())
    cells = ref["sample_cells"]
    for h, r in zip(hist, ref["steps"]):
        assert [int(s) for s in h["sel"]] == r["sel"]
        assert abs(h["E_r"].sum() / r["E_r_sum"] - 1) < 1e-12
        assert abs(h["T"].sum() / r["T_sum"] - 1) < 1e-12
        assert np.allclose(h["E_r"][cells], r["E_r_cells"], rtol=1e-11, atol=0)
        assert np.allclose(h["T"][cells], r["T_cells"], rtol=1e-11, atol=0)
