#!/usr/bin/env python3
"""EPTV iterations/s at 512^2 / 40 views on one MI355X.

One step is one outer iteration of the EPTV algorithm (Sec. 2.2 of the paper):
P1 by CGLS (3 steps: 4 forward projections, 3 backprojections), sigma from the
half-edge magnitudes, P2 by 5 gradient-descent steps with Armijo line search,
positivity.  Workload: 512 x 512 image (1 mm pixels), 40 views over 360 deg,
736-bin equiangular arc detector, SAD 1000 mm, SDD 1500 mm, seeded thorax-like
ellipse phantom with low-contrast inserts, Poisson noise at I0 = 5e4.  Inputs
are resident in HBM before the timed region; the timed region is `--steps`
iterations launched as replays of one captured graph.

Prints one JSON line.  Also measured live: the average duration of the
forward projector and the backprojector (HIP events on their stream) for the
roofline object, and the FP64 CPU oracle on a bounded sample of the same
workload (cpu_baseline).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP32_VECTOR_PEAK = 157.3e12  # MI355X published FP32 vector peak, FLOP/s


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_avg_ms(fn, reps, torch):
    s = torch.cuda.current_stream()
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def cpu_baseline(case, iters):
    import numpy as np
    from oracle import oracle as O

    M = O.Matrix(case.geom)
    p = O.Params(outer_iters=iters, lam=1000.0, tv_eps=1e-4)
    y = case.y.astype(np.float32)
    t0 = time.perf_counter()
    M.reconstruct(y, p)
    dt = time.perf_counter() - t0
    return {"value": iters / dt, "unit": "iterations/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"first {iters} outer iterations of the same 512^2/40-view workload (seed 0), "
                      f"FP64 oracle with a stored Siddon system matrix; matrix build ({M.nnz} nonzeros) "
                      f"excluded like the GPU plan creation",
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--cpu-iters", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only: --gpus {args.gpus} is not supported "
              "(the EPTV path here runs one slice per GPU; slices shard across GPUs without communication)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1009_2288_amd import eptv, synth

    torch.cuda.set_device(0)
    log("bench: building the 512^2 / 40-view case")
    case = synth.make_case("paper", 0)
    g = case.geom
    P = eptv.Plan(g)
    nnz = P.nnz
    y = torch.from_numpy(case.y.astype(np.float32)).cuda()
    ref = torch.from_numpy(case.phantom.astype(np.float32)).cuda()
    f = torch.zeros((g.ny, g.nx), dtype=torch.float32, device="cuda")
    base = dict(cgls_iters=3, tv_iters=5, lam=1000.0, edge_quantile=0.9, tv_eps=1e-4)

    log(f"bench: warmup {args.warmup} iterations")
    P.reconstruct(y, eptv.Params(outer_iters=args.warmup, zero_init=1, **base), f=f, stats=False)
    torch.cuda.synchronize()

    log(f"bench: timing {args.steps} iterations")
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s)
    P.reconstruct(y, eptv.Params(outer_iters=args.steps, zero_init=0, **base), f=f, stats=False)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    its = args.steps / (ms_total / 1e3)
    rmse = float(torch.sqrt(torch.mean((f - ref) ** 2)).item())
    log(f"bench: {its:.1f} it/s ({ms_step:.4f} ms/iteration, wall {wall:.3f} s), rmse {rmse:.3e}")

    # dominant kernels, timed live on the stream they run on
    x = f.clone()
    xT = f.t().contiguous()
    q = P.new_sinogram()
    z = P.new_image()
    r = y.clone()
    t_proj = kernel_avg_ms(lambda: P.project_dual(x, xT, q), args.kernel_reps, torch)
    t_bp = kernel_avg_ms(lambda: P.backproject(r, z), args.kernel_reps, torch)
    per_it = {"project": 4 * t_proj, "backproject": 3 * t_bp}
    dom = max(per_it, key=per_it.get)
    t_dom = t_proj if dom == "project" else t_bp
    flops = 2.0 * nnz
    achieved = flops / (t_dom * 1e-3)
    roof = {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
            "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK, "traffic": None,
            "avg_ms": t_dom, "algorithmic_flops_per_launch": flops, "nnz": nnz,
            "project_avg_ms": t_proj, "backproject_avg_ms": t_bp}
    log(f"bench: project {t_proj * 1e3:.1f} us, backproject {t_bp * 1e3:.1f} us, nnz {nnz}")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"bench: CPU oracle baseline, {args.cpu_iters} iterations")
        cpu = cpu_baseline(case, args.cpu_iters)
        log(f"bench: oracle {cpu['value']:.3f} it/s on {cpu['cores']} threads")

    out = {
        "metric": "EPTV iterations/s at 512^2 / 40 views",
        "value": its,
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "EPTV 512x512 (1 mm), 40 views x 736 bins, SAD 1000 mm, SDD 1500 mm, "
                               "thorax-like ellipse phantom with low-contrast inserts, Poisson I0 5e4; "
                               "per iteration 3 CGLS steps, adaptive sigma (q 0.9), 5 Armijo GD steps, positivity",
                   "image": [g.ny, g.nx], "views": g.n_views, "bins": g.n_bins, "cgls_iters": 3, "tv_iters": 5,
                   "graph": os.environ.get("EPTV_NO_GRAPH", "0") in ("", "0")},
        "rmse_vs_phantom": rmse,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
