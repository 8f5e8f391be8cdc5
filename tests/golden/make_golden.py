"""Write tests/golden/*.json from the FP64 oracle only (no HIP code involved).

Fixtures hold per-step summaries of oracle runs so that an unintended change
of the oracle's arithmetic shows up as a failing regression test.  The paper
prints no numerical worked example, so no fixture here comes from the paper.
Run:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import dlr_oracle as O  # noqa: E402
from synth import problems  # noqa: E402

SAMPLE_CELLS = [0, 5, 31, 100, 333, 512, 777, 1023]


def slab_beam_record():
    p = problems.slab_beam()
    _, hist = O.run_dlr(p)
    steps = []
    for h in hist:
        steps.append({
            "sel": [int(s) for s in h["sel"]],
            "si_iters": int(h["si_iters"]),
            "E_r_sum": float(h["E_r"].sum()),
            "T_sum": float(h["T"].sum()),
            "E_r_cells": [float(h["E_r"][e]) for e in SAMPLE_CELLS],
            "T_cells": [float(h["T"][e]) for e in SAMPLE_CELLS],
            "sigma": [float(s) for s in h["sigma"]],
        })
    return {"problem": p["name"], "sample_cells": SAMPLE_CELLS, "steps": steps,
            "source": "oracle/dlr_oracle.py run_dlr on synth.problems.slab_beam()"}


if __name__ == "__main__":
    rec = slab_beam_record()
    with open(os.path.join(HERE, "slab_beam_32_r8.json"), "w") as f:
        json.dump(rec, f, indent=1)
    print("wrote", rec["problem"])
