"""Writes krylov210.json: the oracle's MMGKS-OF solve with the paper's iteration budget
(Sec. 5: ell = 10 start vectors, up to 200 iterations, flow every 20) on a small moving disk
(synth.cfg_krylov210: 20x20 x 3 frames, 8 angles, 2% noise), so that the last projected
problem has 210 columns; per-iteration RRE, lambda, residual norm and the final u.

Calls only the oracle and the seeded input generators.  Takes about a minute on a CPU:

    python tests/golden/make_krylov210.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mmgks  # noqa: E402
from synth import cfg_krylov210, noisy  # noqa: E402


def main():
    wl = cfg_krylov210()
    s = wl.seqs[0]
    p = wl.params
    prm = {k: p[k] for k in ("ell", "k_max", "tau", "n_sweeps", "alpha", "eps", "eta", "delta_r")}
    g = mmgks.SeqGeom(s.n_t, s.ny, s.nx, s.angles, s.n_bins)
    ops = mmgks.StackOps([g], "radon")
    clean = ops.A(s.u_true.ravel())
    b = noisy(clean, s.noise_g, wl.noise_level)
    delta = float(np.linalg.norm(b - clean))
    ref = mmgks.mmgks_of(ops, b, delta, mmgks.SolveParams(**prm), u_true=s.u_true.ravel())
    out = dict(params=prm, iters=int(ref.iters), n_cols=int(ref.n_cols), rre=[float(x) for x in ref.rre],
               lambdas=[float(x) for x in ref.lambdas], resid=[float(x) for x in ref.resid],
               dp_status=[int(x) for x in ref.dp_status], u=[float(x) for x in ref.u])
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "krylov210.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path, "iters", ref.iters, "n_cols", ref.n_cols, "rre", ref.rre[-1])


if __name__ == "__main__":
    main()
