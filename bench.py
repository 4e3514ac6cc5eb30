#!/usr/bin/env python3
"""EPTV iterations/s at 512^2 / 40 views on one MI355X.

One step is one outer iteration of the EPTV algorithm (Sec. 2.2 of the paper):
P1 by CGLS (3 steps: 4 forward projections, 3 backprojections), sigma from the
half-edge magnitudes, P2 by 5 gradient-descent steps with Armijo line search,
positivity.  Workload: 512 x 512 image (1 mm pixels), 40 views over 360 deg,
736-bin equiangular arc detector, SAD 1000 mm, SDD 1500 mm, seeded thorax-like
ellipse phantom with low-contrast inserts, Poisson noise at I0 = 5e4.  Inputs
are resident in HBM before the timed region; the timed region is `--steps`
iterations, their kernels launched on the stream (the library's default; the
same iterations replayed from a captured graph are timed beside them).

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
HBM_PEAK = 8.0e12            # MI355X published HBM3E bandwidth, B/s
# P and P^T of an outer iteration (the stored_matrix solver parameter):
# on the fly, both from the stored matrix, or P on the fly and P^T stored
OPERATORS = {"fly": 0, "stored": 1, "hybrid": 2}
BF16_MFMA_PEAK = 2.5e15      # MI355X published dense bf16 matrix-core peak, FLOP/s

# HBM bytes per launch of the operator kernels on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each
# scaled by what the counter reads for the read-only stream and a plain device
# copy of known size (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0); see
# profiles/eptv_operators_512x512_40views_pmc_bytes.md.
# Each entry holds the hash of the kernel's source file when the counters were
# taken: if the source has changed since, the figure is stale and reported as
# null.
PMC_TRAFFIC = {
    "project": {"source": "paper_1009_2288_amd/csrc/proj.hip", "sha256_16": "4232d9b9533001f9",
                "bytes": (8343.5 * 2.0 + 125.6 * 1.0) * 1024},
    "backproject": {"source": "paper_1009_2288_amd/csrc/proj.hip", "sha256_16": "4232d9b9533001f9",
                    "bytes": (5979.9 * 2.0 + 1304.0 * 1.0) * 1024},
    "project_stored": {"source": "paper_1009_2288_amd/csrc/spmv.hip", "sha256_16": "fd7c499ef7f7fce8",
                       "bytes": (60465.1 * 2.0 + 129.4 * 1.0) * 1024},
    "backproject_stored": {"source": "paper_1009_2288_amd/csrc/spmv.hip", "sha256_16": "fd7c499ef7f7fce8",
                           "bytes": (56058.5 * 2.0 + 2293.3 * 1.0) * 1024},
}


# The same for the stored products on the paper's scanner at 200 views (the
# stored_hbm leg, whose matrix streams from HBM); see
# profiles/eptv_stored_operators_512x512_200views_paper_scanner_pmc_bytes.md.
PMC_TRAFFIC_HBM = {
    "project_stored": {"source": "paper_1009_2288_amd/csrc/spmv.hip", "sha256_16": "fd7c499ef7f7fce8",
                       "bytes": (426012.5 * 2.0 + 868.4 * 1.0) * 1024},
    "backproject_stored": {"source": "paper_1009_2288_amd/csrc/spmv.hip", "sha256_16": "fd7c499ef7f7fce8",
                           "bytes": (459869.6 * 2.0 + 1193.8 * 1.0) * 1024},
}


# Vector-ALU activity of the operator kernels on this workload from a
# rocprofv3 --pmc pass (VALUBusy, SQ_INSTS_VALU); see
# profiles/eptv_and_unet_valu_mfma_pmc.md.  Reported only while the kernel
# source's hash matches.
PMC_VALU = {
    "project": {"source": "paper_1009_2288_amd/csrc/proj.hip", "sha256_16": "4232d9b9533001f9",
                "valu_busy": 0.404, "valu_wave_instructions": 8.54e6},
    "backproject": {"source": "paper_1009_2288_amd/csrc/proj.hip", "sha256_16": "4232d9b9533001f9",
                    "valu_busy": 0.491, "valu_wave_instructions": 11.47e6},
}


# L2 read bytes per launch (L1-to-L2 read requests x 128-byte lines) from a
# rocprofv3 --pmc pass; see profiles/eptv_operators_512x512_40views_pmc_l2.md.
# Reported only while the kernel source's hash matches.
PMC_L2 = {
    "project": {"source": "paper_1009_2288_amd/csrc/proj.hip", "sha256_16": "4232d9b9533001f9",
                "read_requests": 1.351e6},
    "backproject": {"source": "paper_1009_2288_amd/csrc/proj.hip", "sha256_16": "4232d9b9533001f9",
                    "read_requests": 0.460e6},
    "project_stored": {"source": "paper_1009_2288_amd/csrc/spmv.hip", "sha256_16": "fd7c499ef7f7fce8",
                       "read_requests": 1.517e6},
    "backproject_stored": {"source": "paper_1009_2288_amd/csrc/spmv.hip", "sha256_16": "fd7c499ef7f7fce8",
                           "read_requests": 1.682e6},
}


def pmc_l2(kernel, avg_ms):
    import hashlib
    e = PMC_L2.get(kernel)
    if e is None:
        return None
    with open(os.path.join(ROOT, e["source"]), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest()[:16] != e["sha256_16"]:
            return None
    b = e["read_requests"] * 128.0
    return {"l2_read_bytes_per_launch": b, "l2_read_gbps": b / (avg_ms * 1e-3) / 1e9}


def pmc_valu(kernel, nnz):
    import hashlib
    e = PMC_VALU.get(kernel)
    if e is None:
        return None
    with open(os.path.join(ROOT, e["source"]), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest()[:16] != e["sha256_16"]:
            return None
    return {"valu_busy": e["valu_busy"], "valu_instructions_per_nnz": e["valu_wave_instructions"] * 64 / nnz}


def pmc_traffic(kernel, table=None):
    import hashlib
    e = (PMC_TRAFFIC if table is None else table).get(kernel)
    if e is None:
        return None
    with open(os.path.join(ROOT, e["source"]), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest()[:16] != e["sha256_16"]:
            return None
    return e["bytes"]


def entry_bytes(P, kernel):
    """Stored bytes per nonzero read by a stored-matrix product: a 4-byte
    length with a 16-bit index offset in the compact CSR encoding, else a
    4-byte length and a 4-byte index."""
    return 6.0 if kernel == "project_stored" and P.stored_layout()["csr_compact"] else 8.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def achievable_hbm(torch, mib: int = 2048, reps: int = 10) -> float:
    """Bytes per second of a device-to-device copy of `mib` MiB (read + write)."""
    src = torch.empty(mib * 2**18, dtype=torch.float32, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    sec = a.elapsed_time(b) / 1e3 / reps
    del src, dst
    return 2.0 * mib * 2**20 / sec


def achievable_read(torch, eptv, mib: int = 2048, reps: int = 10) -> float:
    """Bytes per second of the library's read-only streaming kernel over a
    `mib` MiB buffer, far larger than the 256 MB Infinity Cache: the rate a
    read-dominated kernel can reach from HBM on this GPU."""
    buf = torch.empty(mib * 2**18, dtype=torch.float32, device="cuda").fill_(1.0)
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    ms = kernel_avg_ms(lambda: eptv.stream_read(buf, sink), reps, torch)
    del buf
    return mib * 2**20 / (ms * 1e-3)


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


def host_cpu():
    """The host CPU: model name, logical CPUs, physical cores (distinct
    (package, core) pairs in /proc/cpuinfo) and the CPUs this process may use."""
    model, logical, cores, cur = None, 0, set(), {}
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in list(fh) + [""]:
                if not ln.strip():
                    if "processor" in cur:
                        logical += 1
                        cores.add((cur.get("physical id"), cur.get("core id")))
                        model = model or cur.get("model name")
                    cur = {}
                    continue
                k, _, v = ln.partition(":")
                cur[k.strip()] = v.strip()
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        allowed = os.cpu_count()
    return {"model": model, "logical_cpus": logical or None, "physical_cores": len(cores) or None,
            "cpus_available": allowed}


def cpu_baseline(cases, iters_n, iters_1, small_iters):
    """The FP64 oracle as it stands, on this host: the 512^2/40-view workload
    (iters_n outer iterations on all available CPUs, iters_1 on one thread) and
    the 128^2/30-view one (small_iters each way), matrix builds excluded like
    the GPU plan creation; one oracle call of P and P^T at each thread count.
    value: the 512^2 iterations per second on all available CPUs."""
    import numpy as np
    from oracle import oracle as O

    cpu = host_cpu()
    n_threads = max(1, int(cpu["cpus_available"] or 1))
    runs = {}
    for name, case, iters in (("paper", cases["paper"], (iters_n, iters_1)),
                              ("small", cases["small"], (small_iters, small_iters))):
        M = O.Matrix(case.geom)
        y = case.y.astype(np.float32)
        x = case.phantom.astype(np.float32)
        for threads, k in ((n_threads, iters[0]), (1, iters[1])):
            if k <= 0:
                continue
            O.set_num_threads(threads)
            t0 = time.perf_counter()
            M.reconstruct(y, O.Params(outer_iters=k, lam=1000.0, tv_eps=1e-4))
            dt = time.perf_counter() - t0
            t1 = time.perf_counter()
            M.project(x)
            t2 = time.perf_counter()
            M.backproject(y)
            t3 = time.perf_counter()
            runs[f"{name}_{'1' if threads == 1 else 'n'}"] = {
                "threads": O.num_threads(), "iterations": k, "seconds": dt, "iterations_per_s": k / dt,
                "project_ms": (t2 - t1) * 1e3, "backproject_ms": (t3 - t2) * 1e3, "nnz": M.nnz}
    O.set_num_threads(n_threads)
    head = runs["paper_n"]
    return {"value": head["iterations_per_s"], "unit": "iterations/s", "cores": head["threads"], "kind": "oracle",
            "sample": f"the first {iters_n} outer iterations of the same 512^2/40-view workload (seed 0) on "
                      f"{head['threads']} threads, FP64 oracle with a stored Siddon system matrix; matrix build "
                      f"excluded like the GPU plan creation; beside it {iters_1} iterations on one thread and "
                      f"{small_iters} iterations of the 128^2/30-view workload each way",
            "seconds": head["seconds"], "project_ms": head["project_ms"], "backproject_ms": head["backproject_ms"],
            "cpu": cpu, "runs": runs}


def time_to_rmse(E, synth, P, torch, np, seeds, solver):
    """Seconds until the RMSE to the phantom reaches a target of the FP64
    oracle's (tests/golden/rmse_targets_paper.json), the device-side RMSE
    record included in the timed run; per seed the median of repeated runs,
    over seeds the median.  Targets: the oracle's RMSE after 100 iterations,
    and (stricter) its best RMSE over those iterations plus 0.1 % (the float32
    trajectory follows the oracle's to ~1e-5, so its minimum may sit a hair
    above).  Plain EPTV from zero, and (when the trained network is present)
    the CNN-assisted pipeline: plain iterations (1), the U-Net's proposal of
    image and edge weights, EPTV warm-started from it with the weights frozen
    for its first iteration."""
    from paper_1009_2288_amd import cnn_assist as A
    with open(os.path.join(ROOT, "tests", "golden", "rmse_targets_paper.json")) as fh:
        targets = json.load(fh)
    net = A.network(max_batch=1, params=A.load_params()) if os.path.exists(A.WEIGHTS) else None
    per = []
    for seed in seeds:
        c = synth.make_case("paper", seed)
        y = torch.from_numpy(c.y.astype(np.float32)).cuda()
        ref = torch.from_numpy(c.phantom.astype(np.float32)).cuda()
        t_final = targets["seeds"][str(seed)]["rmse_final"]
        t_min = targets["seeds"][str(seed)]["rmse_min"] * 1.001
        r = {"seed": seed, "target": t_final, "target_min": t_min,
             "plain": A.time_to_rmse(P, y, ref, t_final, solver=solver),
             "plain_min": A.time_to_rmse(P, y, ref, t_min, solver=solver)}
        if net is not None:
            r["cnn"] = A.time_to_rmse(P, y, ref, t_final, net=net, solver=solver)
            r["cnn_min"] = A.time_to_rmse(P, y, ref, t_min, net=net, solver=solver)
        per.append(r)

    def med(kind, key):
        v = [p[kind][key] for p in per if kind in p]
        return float(np.median(v)) if v and all(x is not None for x in v) else None

    out = {"target": "FP64 oracle RMSE to the phantom after 100 iterations, same seed",
           "target_min": "FP64 oracle's best RMSE over its 100 iterations (about iteration 27) + 0.1 %, same seed",
           "plain_seconds_median": med("plain", "seconds"),
           "plain_iterations_median": med("plain", "iterations"),
           "plain_min_seconds_median": med("plain_min", "seconds"),
           "plain_min_iterations_median": med("plain_min", "iterations"),
           "per_seed": per}
    if net is not None:
        out["cnn_seconds_median"] = med("cnn", "seconds")
        out["cnn_warm_iterations_median"] = med("cnn", "iterations")
        out["cnn_min_seconds_median"] = med("cnn_min", "seconds")
        out["cnn_min_warm_iterations_median"] = med("cnn_min", "iterations")
        if out["cnn_seconds_median"] and out["plain_seconds_median"]:
            out["cnn_speedup"] = out["plain_seconds_median"] / out["cnn_seconds_median"]
        if out["cnn_min_seconds_median"] and out["plain_min_seconds_median"]:
            out["cnn_min_speedup"] = out["plain_min_seconds_median"] / out["cnn_min_seconds_median"]
        out["cnn_pipeline"] = (f"{A.N0} plain iterations + U-Net ({A.NET['levels']} levels, base {A.NET['base']}, "
                               f"bf16 MFMA) + EPTV warm start, proposed weights frozen for 1 iteration")
        # the network alone: forward time and matrix-core rate at 512^2
        x = torch.zeros((1, 512, 512, 1), dtype=torch.float32, device="cuda")
        for _ in range(3):
            net.forward(x)
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        for _ in range(20):
            net.forward(x)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 20
        fl = A.forward_flops(512, 512)
        out["unet_forward"] = {"ms": ms, "algorithmic_gflop": fl / 1e9, "tflops": fl / ms / 1e9,
                               "mfma_bf16_peak_frac": fl / (ms * 1e-3) / BF16_MFMA_PEAK}
    return out


def unet_training_leg(torch, np, steps, batch=8):
    """Training throughput of the EPTV-assist U-Net (4 levels, base 32, 512^2)
    on the library's kernels: forward, MSE, backward, Adam per step, batch 8;
    inputs are random (the kernels' work does not depend on the values)."""
    from paper_1009_2288_amd import cnn_assist as A
    net = A.network(max_batch=batch)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    x = torch.randn((batch, 512, 512, 1), generator=g, device="cuda")
    t = torch.randn((batch, 512, 512, 3), generator=g, device="cuda")

    def step(i):
        y = net.forward(x)
        _, dy = net.mse(y, t)
        net.backward(dy)
        net.adam(1e-4, i + 1)

    step(0)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for i in range(steps):
        step(i + 1)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    fl = 3.0 * A.forward_flops(512, 512) * batch  # forward + data gradient + weight gradient
    return {"batch": batch, "steps": steps, "ms_per_step": ms, "images_per_s": batch * 1e3 / ms,
            "algorithmic_tflops": fl / ms / 1e9, "mfma_bf16_peak_frac": fl / (ms * 1e-3) / BF16_MFMA_PEAK}


def batch_leg(E, synth, torch, np, n_slices, iters, warmup):
    """The batched workload: n_slices slices of 256^2 / 384^2 / 512^2, 20-60
    views, 368-736 bins, I0 1e4-1e5 (seed 0), every phase one launch over all
    slices (launched on the stream like the one-slice path), launch shapes
    from the tuner."""
    cases = synth.batch_cases(n_slices, 0, with_phantom=False)
    B = E.Batch([c.geom for c in cases])
    tuned = B.tune(reps=5)
    ys = [torch.from_numpy(c.y.astype(np.float32)).cuda() for c in cases]
    prm = dict(cgls_iters=3, tv_iters=5, lam=1000.0, edge_quantile=0.9, tv_eps=1e-4)
    fs, _ = B.reconstruct(ys, E.Params(outer_iters=warmup, zero_init=1, **prm), stats=False)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    B.reconstruct(ys, E.Params(outer_iters=iters, zero_init=0, **prm), fs=fs, stats=False)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    work = sum(c.geom.nx * c.geom.ny * c.geom.n_views for c in cases) / (512 * 512 * 40)
    return {"slices": n_slices, "iterations": iters, "ms_per_batch_iteration": ms,
            "slice_iterations_per_s": n_slices * 1e3 / ms,
            "work_in_512x512x40_slices": work,
            "equivalent_512x512x40_iterations_per_s": work * 1e3 / ms,
            "launch": tuned,
            "workload": "64 seeded slices, side uniform in {256, 384, 512} (1 mm), views 20-60, bins 368-736, "
                        "I0 log-uniform 1e4-1e5; per iteration 3 CGLS steps, adaptive sigma, 5 Armijo steps"}


def paper_scanner_geometry(synth, n_views):
    """The paper's scanner (Sec. 3): an 888-unit arc detector at 1.0239 mm
    pitch and 949.075 mm from the source, 541 mm from source to rotation
    centre, a 512 x 512 image whose inscribed circle is the fan's field of view
    (0.974 mm pixels; the corners lie outside the fan, as on a clinical
    scanner)."""
    import math
    dbeta = 1.0239 / 949.075
    pixel = 2.0 * 541.0 * math.sin(0.5 * 888 * dbeta) / 512
    return synth.Geometry(512, 512, pixel, n_views, 888, dbeta, 541.0, 949.075)


def stored_hbm_leg(E, synth, torch, np, reps, steps, n_views=200):
    """The stored-matrix products (the paper's look-up tables, Sec. 2.3) on a
    workload whose two copies exceed the 256 MB Infinity Cache, so every call
    streams them from HBM: the paper's scanner at the chest case's 200 views
    (Table 2).  Per-call kernel times (HIP events on the launching stream)
    against the algorithmic bytes, the read-only streaming rate of this GPU,
    and whole EPTV iterations at this size with each operator mode."""
    g = paper_scanner_geometry(synth, n_views)
    ell = synth.phantom_paper(0)
    y_np = synth.noisy_sinogram(synth.line_integrals(ell, g), 5e4, 1000).astype(np.float32)
    P = E.Plan(g)
    nnz = P.nnz
    mbytes = P.store_matrix()
    y = torch.from_numpy(y_np).cuda()
    x = torch.rand((g.ny, g.nx), generator=torch.Generator(device="cuda").manual_seed(1), device="cuda")
    xT = x.t().contiguous()
    q = P.new_sinogram()
    z = P.new_image()
    n_img, n_sino = g.nx * g.ny, g.n_views * g.n_bins
    out = {"workload": f"the paper's scanner: 512x512 ({g.pixel_mm:.3f} mm pixels), {n_views} views x 888 bins, "
                       f"SAD 541 mm, SDD 949.075 mm (the chest case of Table 2)",
           "nnz": nnz, "matrix_bytes": mbytes}
    for name, fn, rows, n_in, n_out in (
            ("project_stored", lambda: P.project_stored_dual(x, xT, q), n_sino, n_img, n_sino),
            ("backproject_stored", lambda: P.backproject_stored(y, z), n_img, n_sino, n_img)):
        ms = kernel_avg_ms(fn, reps, torch)
        nbytes = entry_bytes(P, name) * nnz + 4.0 * (rows + 1) + 4.0 * (n_in + n_out)
        out[name] = {"avg_ms": ms, "algorithmic_bytes_per_launch": nbytes, "gbps": nbytes / (ms * 1e-3) / 1e9,
                     "frac": nbytes / (ms * 1e-3) / HBM_PEAK}
    rd = achievable_read(torch, E)
    out["achievable_read_gbps"] = rd / 1e9
    for name in ("project_stored", "backproject_stored"):
        out[name]["frac_of_achievable"] = out[name]["gbps"] * 1e9 / rd
        out[name]["traffic"] = pmc_traffic(name, PMC_TRAFFIC_HBM)
    # the roofline object for this workload's dominant stored kernel (4 P and
    # 3 P^T calls per outer iteration)
    dom = max(("project_stored", "backproject_stored"),
              key=lambda k: (4 if k == "project_stored" else 3) * out[k]["avg_ms"])
    d = out[dom]
    out["roofline"] = {"bound": "hbm", "kernel": dom, "achieved": d["gbps"], "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                       "frac": d["frac"], "traffic": d["traffic"], "avg_ms": d["avg_ms"],
                       "algorithmic_bytes_per_launch": d["algorithmic_bytes_per_launch"],
                       "frac_of_achievable": d["frac_of_achievable"]}
    its = {}
    base = dict(cgls_iters=3, tv_iters=5, lam=1000.0, edge_quantile=0.9, tv_eps=1e-4)
    for mode in ("stored", "fly", "hybrid"):
        prm = dict(base, stored_matrix=OPERATORS[mode])
        f = torch.zeros((g.ny, g.nx), dtype=torch.float32, device="cuda")
        P.reconstruct(y, E.Params(outer_iters=2, zero_init=1, **prm), f=f, stats=False)
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s)
        P.reconstruct(y, E.Params(outer_iters=steps, zero_init=0, **prm), f=f, stats=False)
        e1.record(s)
        torch.cuda.synchronize()
        its[mode] = steps / (e0.elapsed_time(e1) / 1e3)
    out["iterations_per_s"] = its
    out["paper_context"] = "Table 2, chest: 200 views, 30 iterations in 9.8 s on a Tesla C1060 (0.327 s per iteration)"
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--cpu-iters", type=int, default=60,
                    help="outer iterations of the FP64 oracle on all host CPUs for cpu_baseline (512^2/40 views)")
    ap.add_argument("--cpu-iters-1", type=int, default=20,
                    help="outer iterations of the FP64 oracle on one thread (512^2/40 views)")
    ap.add_argument("--cpu-small-iters", type=int, default=50,
                    help="outer iterations of the FP64 oracle on the 128^2/30-view workload, each thread count")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--rmse-seeds", type=int, default=10, help="seeds for the time-to-RMSE leg (0 to skip)")
    ap.add_argument("--batch-slices", type=int, default=64, help="slices of the batched leg (0 to skip)")
    ap.add_argument("--batch-iters", type=int, default=20)
    ap.add_argument("--unet-train-steps", type=int, default=10,
                    help="timed training steps of the EPTV-assist U-Net (0 to skip)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="finally copy a buffer of this many MiB on the device (a plain copy kernel of known "
                         "size, to calibrate hardware byte counters against)")
    ap.add_argument("--hbm-views", type=int, default=200,
                    help="views of the stored-matrix leg on the paper's scanner, whose matrix streams from HBM "
                         "(0 to skip)")
    ap.add_argument("--operator", choices=list(OPERATORS), default="stored",
                    help="P and P^T of the headline figure: from the stored float32 matrix (the paper's "
                         "look-up tables), on the fly, or P on the fly with P^T stored (hybrid); the others "
                         "are timed and reported beside it")
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
    log(f"bench: storing the system matrix ({P.store_matrix() / 2**20:.0f} MiB)")
    base = dict(cgls_iters=3, tv_iters=5, lam=1000.0, edge_quantile=0.9, tv_eps=1e-4)

    def iterations(mode):
        """Iterations/s of `args.steps` outer iterations after `args.warmup`."""
        prm = dict(base, stored_matrix=OPERATORS[mode])
        f = torch.zeros((g.ny, g.nx), dtype=torch.float32, device="cuda")
        P.reconstruct(y, eptv.Params(outer_iters=args.warmup, zero_init=1, **prm), f=f, stats=False)
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record(s)
        P.reconstruct(y, eptv.Params(outer_iters=args.steps, zero_init=0, **prm), f=f, stats=False)
        e1.record(s)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms_total = e0.elapsed_time(e1)
        rmse = float(torch.sqrt(torch.mean((f - ref) ** 2)).item())
        log(f"bench: {mode}: {args.steps / (ms_total / 1e3):.1f} it/s ({ms_total / args.steps:.4f} ms/iteration, "
            f"wall {wall:.3f} s), rmse {rmse:.3e}")
        return args.steps / (ms_total / 1e3), ms_total / args.steps, rmse, f

    log(f"bench: warmup {args.warmup}, timing {args.steps} iterations per operator")
    its, ms_step, rmse, f = iterations(args.operator)
    others = {m: iterations(m)[:3] for m in OPERATORS if m != args.operator}
    # the headline operator once more with the other launch mode (graph replay
    # if the headline launched its kernels directly, and the reverse)
    had = os.environ.get("EPTV_GRAPH")
    headline_graph = had not in (None, "", "0")
    os.environ["EPTV_GRAPH"] = "0" if headline_graph else "1"
    try:
        its_ng, ms_ng, _, _ = iterations(args.operator)
    finally:
        if had is None:
            os.environ.pop("EPTV_GRAPH", None)
        else:
            os.environ["EPTV_GRAPH"] = had

    # dominant kernels, timed live on the stream they run on
    x = f.clone()
    xT = f.t().contiguous()
    q = P.new_sinogram()
    z = P.new_image()
    r = y.clone()
    ops = {"project_dual": lambda: P.project_dual(x, xT, q), "backproject": lambda: P.backproject(r, z),
           "backproject_interp": lambda: P.backproject_interp(r, z),
           "project_stored": lambda: P.project_stored_dual(x, xT, q),
           "backproject_stored": lambda: P.backproject_stored(r, z)}
    op_ms = {k: kernel_avg_ms(fn, args.kernel_reps, torch) for k, fn in ops.items()}
    log("bench: " + ", ".join(f"{k} {v * 1e3:.1f} us" for k, v in op_ms.items()) + f", nnz {nnz}")

    def roofline(mode):
        # the operator kernels of an outer iteration: 4 P calls and 3 P^T calls
        k_proj = "project_stored" if mode == "stored" else "project_dual"
        k_bp = "backproject" if mode == "fly" else "backproject_stored"
        per_it = {"project": 4 * op_ms[k_proj], "backproject": 3 * op_ms[k_bp]}
        dom = max(per_it, key=per_it.get)
        kern = k_proj if dom == "project" else k_bp
        t_dom = op_ms[kern]
        if kern.endswith("_stored"):
            # one CSR (or CSC) pass: each nonzero at its stored size (see
            # entry_bytes; the padding to 4 entries per row and the CSR chunk
            # bases are overhead, not counted), a 4-byte offset per row
            # (column), the input vector once, the output once
            n_img, n_sino = g.nx * g.ny, g.n_views * g.n_bins
            rows, n_in, n_out = (n_sino, n_img, n_sino) if dom == "project" else (n_img, n_sino, n_img)
            nbytes = entry_bytes(P, dom + "_stored") * nnz + 4.0 * (rows + 1) + 4.0 * (n_in + n_out)
            achieved = nbytes / (t_dom * 1e-3)
            return {"bound": "hbm", "kernel": dom + "_stored", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK, "traffic": pmc_traffic(dom + "_stored"),
                    "avg_ms": t_dom, "algorithmic_bytes_per_launch": nbytes, "nnz": nnz,
                    "pmc_l2": pmc_l2(dom + "_stored", t_dom)}
        flops = 2.0 * nnz
        achieved = flops / (t_dom * 1e-3)
        return {"bound": "alu", "kernel": dom, "achieved": achieved / 1e12, "peak": FP32_VECTOR_PEAK / 1e12,
                "unit": "TFLOP/s", "frac": achieved / FP32_VECTOR_PEAK, "traffic": pmc_traffic(dom),
                "avg_ms": t_dom, "algorithmic_flops_per_launch": flops, "nnz": nnz,
                "pmc_valu": pmc_valu(dom, nnz), "pmc_l2": pmc_l2(dom, t_dom)}

    roof = roofline(args.operator)
    roof["operators_avg_ms"] = op_ms
    other = [{"operator": m, "stored_matrix": OPERATORS[m], "value": v[0], "ms_per_step": v[1],
              "rmse_vs_phantom": v[2], "roofline": roofline(m)} for m, v in others.items()]
    if roof["bound"] == "hbm":
        # what HBM delivers to a read-only stream and to a device copy, both far
        # larger than the 256 MB Infinity Cache; at this size the two matrix
        # copies (together under 256 MB) are served partly by that cache between
        # calls, so the fraction is cache-assisted (stored_hbm streams them)
        rd = achievable_read(torch, eptv)
        roof["achievable_read_gbps"] = rd / 1e9
        roof["frac_of_achievable"] = roof["achieved"] * 1e9 / rd
        roof["achievable_copy_gbps"] = achievable_hbm(torch) / 1e9
        roof["note"] = ("cache-assisted: both stored copies (%.0f MB) fit the 256 MB Infinity Cache between calls"
                        % (P.store_matrix() / 1e6))
        if roof["kernel"] == "project_stored" and P.stored_layout()["csr_compact"]:
            roof["note"] += ("; P reads the compact CSR encoding (6 bytes per nonzero, the bytes counted here; "
                             "the same call at 8 bytes per nonzero would be %.0f GB/s)"
                             % (roof["achieved"] * (roof["algorithmic_bytes_per_launch"] + 2.0 * nnz)
                                / roof["algorithmic_bytes_per_launch"]))
    log("bench: " + ", ".join(f"{k} {v * 1e3:.1f} us" for k, v in op_ms.items()) + f", nnz {nnz}")

    ttr = None
    if args.rmse_seeds > 0:
        log(f"bench: time to the oracle's RMSE, seeds 0-{args.rmse_seeds - 1}")
        ttr = time_to_rmse(eptv, synth, P, torch, np, range(args.rmse_seeds), {"stored_matrix": OPERATORS[args.operator]})
        log(f"bench: plain EPTV reaches the oracle RMSE in {ttr['plain_seconds_median']} s (median), "
            f"CNN-assisted in {ttr.get('cnn_seconds_median')} s")

    bat = None
    if args.batch_slices > 0:
        log(f"bench: batched leg, {args.batch_slices} slices")
        bat = batch_leg(eptv, synth, torch, np, args.batch_slices, args.batch_iters, 3)
        log(f"bench: batch {bat['ms_per_batch_iteration']:.3f} ms per iteration of all slices, "
            f"{bat['equivalent_512x512x40_iterations_per_s']:.1f} equivalent 512^2/40 it/s, launch {bat['launch']}")

    hbm_leg = None
    if args.hbm_views > 0:
        log(f"bench: stored matrix streaming from HBM, the paper's scanner at {args.hbm_views} views")
        hbm_leg = stored_hbm_leg(eptv, synth, torch, np, max(10, args.kernel_reps // 10), 10, args.hbm_views)
        log(f"bench: stored P {hbm_leg['project_stored']['gbps']:.0f} GB/s, P^T "
            f"{hbm_leg['backproject_stored']['gbps']:.0f} GB/s, read stream {hbm_leg['achievable_read_gbps']:.0f} "
            f"GB/s, matrix {hbm_leg['matrix_bytes'] / 2**20:.0f} MiB, it/s {hbm_leg['iterations_per_s']}")

    cnn_train = None
    if args.unet_train_steps > 0:
        log(f"bench: U-Net training, {args.unet_train_steps} steps of batch 8")
        cnn_train = unet_training_leg(torch, np, args.unet_train_steps)
        log(f"bench: U-Net training {cnn_train['ms_per_step']:.2f} ms per step, "
            f"{cnn_train['algorithmic_tflops']:.0f} TFLOP/s")

    cpu = None
    if not args.no_cpu_baseline:
        log(f"bench: CPU oracle baseline, {args.cpu_iters} + {args.cpu_iters_1} iterations (512^2), "
            f"{args.cpu_small_iters} x 2 (128^2)")
        cpu = cpu_baseline({"paper": case, "small": synth.make_case("small", 0)}, args.cpu_iters, args.cpu_iters_1,
                           args.cpu_small_iters)
        log(f"bench: oracle {cpu['value']:.3f} it/s on {cpu['cores']} threads; "
            + ", ".join(f"{k} {v['iterations_per_s']:.3f} it/s" for k, v in cpu["runs"].items()))

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
                   "graph": headline_graph, "operator": args.operator},
        "rmse_vs_phantom": rmse,
        "other_operators": other,
        ("without_graph" if headline_graph else "with_graph"): {
            "value": its_ng, "ms_per_step": ms_ng,
            "note": ("same operator, each of the iteration's kernels launched on the stream" if headline_graph
                     else "same operator, the iteration captured once as a HIP graph and replayed")},
        "time_to_rmse": ttr,
        "batch": bat,
        "stored_hbm": hbm_leg,
        "cnn_training": cnn_train,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib * 2**18, dtype=torch.float32, device="cuda")
        dst = src.clone()
        torch.cuda.synchronize()
        log(f"bench: copied {args.copy_mib} MiB ({float(dst[-1]):.0f})")


if __name__ == "__main__":
    main()
