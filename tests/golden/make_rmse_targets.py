"""Writes rmse_targets_paper.json: the FP64 oracle's RMSE to the phantom after
100 EPTV iterations on the 512^2 / 40-view workload, seeds 0-9.

These are the targets of the time-to-RMSE measurement (plain EPTV on the GPU
runs until its RMSE reaches the oracle's).  Only the oracle and the seeded
input generator are called.  Run from the repository root:

    python tests/golden/make_rmse_targets.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1009_2288_amd import synth  # noqa: E402

ITERS = 100
PARAMS = dict(cgls_iters=3, tv_iters=5, lam=1000.0, edge_quantile=0.9, tv_eps=1e-4)


def main():
    out = {"workload": "512x512 (1 mm), 40 views x 736 bins, SAD 1000, SDD 1500, I0 5e4",
           "iterations": ITERS, "params": PARAMS, "seeds": {}}
    M = None
    for seed in range(10):
        c = synth.make_case("paper", seed)
        if M is None:
            M = O.Matrix(c.geom)
        _, st = M.reconstruct(c.y.astype(np.float32), O.Params(outer_iters=ITERS, **PARAMS), f_ref=c.phantom)
        r = st["rmse"]
        out["seeds"][str(seed)] = {"rmse_final": float(r[-1]), "rmse_min": float(r.min()),
                                   "iter_min": int(r.argmin()) + 1}
        print(seed, out["seeds"][str(seed)], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "rmse_targets_paper.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
