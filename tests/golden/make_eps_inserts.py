"""Writes eps_inserts_paper.json: how the eps of Eq. A3 (the floor under the
half-edge magnitudes, which A2's fluxes divide by) affects the low-contrast
inserts of the 512^2 / 40-view workload, computed by the FP64 oracle.

EPTV's weights (Eq. 5) are meant to spare edges from smoothing (Sec. 2.1);
with eps comparable to an edge's jump the edge's magnitude is dominated by eps
and its flux becomes linear in the difference.  The inserts' contrasts are
1e-4 to 4e-4 mm^-1, the low end equal to the library's default eps = 1e-4.
For eps = 1e-4 and 1e-6, seeds 0-4, after 27 iterations (about where the
oracle's whole-image RMSE is lowest) and after 100, per insert:
  * contrast recovery: (mean over the disc shrunk by 2 mm - mean over the ring
    3-6 mm outside it) / the insert's true contrast;
  * ROI RMSE: RMSE to the phantom raster over the disc grown by 2 mm (its
    edge included).
Only the oracle and the seeded input generator are called.  Run from the
repository root:

    python tests/golden/make_eps_inserts.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1009_2288_amd import synth  # noqa: E402

SEEDS = range(5)
EPS = (1e-4, 1e-6)
CHECKPOINTS = (27, 100)
PARAMS = dict(cgls_iters=3, tv_iters=5, lam=1000.0, edge_quantile=0.9)


def insert_masks(e, g):
    xs = (np.arange(g.nx) + 0.5 - 0.5 * g.nx) * g.pixel_mm
    ys = (np.arange(g.ny) + 0.5 - 0.5 * g.ny) * g.pixel_mm
    X, Y = np.meshgrid(xs, ys)
    d = np.hypot(X - e.cx, Y - e.cy)
    r = e.a
    return d <= r - 2.0, (d >= r + 3.0) & (d <= r + 6.0), d <= r + 2.0


def measure(f, c, ell):
    out = []
    for e in ell:
        inner, ring, roi = insert_masks(e, c.geom)
        rec = (f[inner].mean() - f[ring].mean()) / e.mu
        rmse = float(np.sqrt(np.mean((f[roi] - c.phantom[roi]) ** 2)))
        out.append({"contrast": e.mu, "radius_mm": e.a, "recovery": float(rec), "roi_rmse": rmse})
    return out


def main():
    res = {"workload": "512x512 (1 mm), 40 views x 736 bins, SAD 1000, SDD 1500, I0 5e4", "params": PARAMS,
           "checkpoints": list(CHECKPOINTS), "runs": {}}
    M = None
    for seed in SEEDS:
        c = synth.make_case("paper", seed)
        low = synth.phantom_paper(seed)[-6:]  # the six low-contrast discs
        if M is None:
            M = O.Matrix(c.geom)
        y = c.y.astype(np.float32)
        for eps in EPS:
            f = np.zeros((c.geom.ny, c.geom.nx))
            done, per = 0, {}
            for k in CHECKPOINTS:
                f, st = M.reconstruct(y, O.Params(outer_iters=k - done, zero_init=int(done == 0), tv_eps=eps,
                                                  **PARAMS), f0=f, f_ref=c.phantom)
                done = k
                per[str(k)] = {"rmse": float(st["rmse"][-1]), "inserts": measure(f, c, low)}
            res["runs"][f"seed{seed}_eps{eps:g}"] = per
            rec = np.mean([i["recovery"] for i in per["27"]["inserts"]])
            print(seed, eps, per["27"]["rmse"], per["100"]["rmse"], f"mean recovery @27 {rec:.3f}", flush=True)
    # summary: per eps and checkpoint, the mean over inserts and seeds
    summ = {}
    for eps in EPS:
        for k in CHECKPOINTS:
            ins = [i for s in SEEDS for i in res["runs"][f"seed{s}_eps{eps:g}"][str(k)]["inserts"]]
            weak = [i for i in ins if abs(i["contrast"]) <= 2e-4]
            summ[f"eps{eps:g}_iter{k}"] = {
                "image_rmse_mean": float(np.mean([res["runs"][f"seed{s}_eps{eps:g}"][str(k)]["rmse"] for s in SEEDS])),
                "recovery_mean": float(np.mean([i["recovery"] for i in ins])),
                "recovery_mean_weakest": float(np.mean([i["recovery"] for i in weak])) if weak else None,
                "n_weakest": len(weak),
                "roi_rmse_mean": float(np.mean([i["roi_rmse"] for i in ins]))}
    res["summary"] = summ
    print(json.dumps(summ, indent=1))
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "eps_inserts_paper.json"), "w") as fh:
        json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
