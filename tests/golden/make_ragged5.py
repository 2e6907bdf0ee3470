"""Writes ragged5.json: the oracle's MMGKS-OF solve of a ragged batch taken from the batched
deblurring workload (synth.cfg_blur_ragged): its five smallest sequences (80^2 x 8, 98^2 x 9,
71^2 x 9, 115^2 x 12, 70^2 x 14 frames; rotating ellipses, 9x9 Gaussian blur sigma 2, 1% noise
over the five), solved as one problem with the workload's settings (ell 10, flow every 10 with
100 Horn-Schunck sweeps, alpha 0.1) for 13 outer iterations, so one flow update on a nonzero
image is included; per-iteration lambda, residual norm and RRE.

Calls only the oracle and the seeded input generators.  Takes about a minute on a CPU:

    python tests/golden/make_ragged5.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import mmgks  # noqa: E402
from synth import cfg_blur_ragged, noisy  # noqa: E402

K_MAX = 13


def subset():
    """The workload, the indices of its five smallest sequences (in stack order) and the data."""
    wl = cfg_blur_ragged()
    order = sorted(range(len(wl.seqs)), key=lambda i: wl.seqs[i].u_true.size)
    pick = sorted(order[:5])
    seqs = [wl.seqs[i] for i in pick]
    geoms = [mmgks.SeqGeom(s.n_t, s.ny, s.nx, ksize=9, sigma=2.0) for s in seqs]
    ops = mmgks.StackOps(geoms, "blur")
    ut = np.concatenate([s.u_true.ravel() for s in seqs])
    clean = ops.A(ut)
    b = noisy(clean, np.concatenate([s.noise_g.ravel() for s in seqs]), wl.noise_level)
    return wl, pick, seqs, ops, ut, b, float(np.linalg.norm(b - clean))


def main():
    wl, pick, seqs, ops, ut, b, delta = subset()
    p = wl.params
    prm = dict(ell=p["ell"], k_max=K_MAX, tau=p["tau"], n_sweeps=p["n_sweeps"], alpha=p["alpha"], eps=p["eps"],
               eta=p["eta"], delta_r=p["delta_r"])
    ref = mmgks.mmgks_of(ops, b, delta, mmgks.SolveParams(**prm), u_true=ut)
    out = dict(pick=pick, sizes=[[s.n_t, s.ny, s.nx] for s in seqs], params=prm, iters=int(ref.iters),
               rre=[float(x) for x in ref.rre], lambdas=[float(x) for x in ref.lambdas],
               resid=[float(x) for x in ref.resid], dp_status=[int(x) for x in ref.dp_status])
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ragged5.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, "rre", ref.rre[-1])


if __name__ == "__main__":
    main()
