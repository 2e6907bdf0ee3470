"""Writes solve_ellipse128.json: the oracle's MMGKS-OF solve of the 128x128x16 moving-ellipse
workload (30 angles per frame, 181 bins, 2% noise; ell 10, 30 outer iterations, flow update
every 10, 200 Horn-Schunck sweeps, alpha 0.1), per-iteration RRE, lambda and residual norm.

Calls only the oracle and the seeded input generators.  Takes a few minutes on a CPU:

    python tests/golden/make_solve_ellipse128.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mmgks  # noqa: E402
from synth import cfg_ellipse128, noisy  # noqa: E402

PARAMS = dict(ell=10, k_max=30, tau=10, n_sweeps=200, alpha=0.1, eps=1e-3, eta=1.01, delta_r=1)


def main():
    wl = cfg_ellipse128()
    s = wl.seqs[0]
    g = mmgks.SeqGeom(s.n_t, s.ny, s.nx, s.angles, s.n_bins)
    ops = mmgks.StackOps([g], "radon")
    clean = ops.A(s.u_true.ravel())
    b = noisy(clean, s.noise_g, wl.noise_level)
    delta = float(np.linalg.norm(b - clean))
    ref = mmgks.mmgks_of(ops, b, delta, mmgks.SolveParams(**PARAMS), u_true=s.u_true.ravel())
    out = dict(params=PARAMS, iters=int(ref.iters), rre=[float(x) for x in ref.rre],
               lambdas=[float(x) for x in ref.lambdas], resid=[float(x) for x in ref.resid],
               dp_status=[int(x) for x in ref.dp_status])
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "solve_ellipse128.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
