"""Size bookkeeping of the stacked operators against the sizes the paper prints."""
import json
import os

import numpy as np

from oracle import mmgks

HERE = os.path.dirname(os.path.abspath(__file__))


def test_paper_operator_sizes():
    with open(os.path.join(HERE, "golden", "paper_sizes.json")) as f:
        cases = json.load(f)["cases"]
    for c in cases:
        ang = np.zeros((c["n_t"], c["n_theta"]))
        g = mmgks.SeqGeom(c["n_t"], c["ny"], c["nx"], ang, c["n_bins"])
        ops = mmgks.StackOps([g], "radon")
        assert (ops.m, ops.n) == (c["m"], c["n"]), c["cite"]
