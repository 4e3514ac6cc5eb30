"""The batched EPTV iteration on the GPU: every phase one launch over all
slices.  A slice of a batch must get exactly what it gets alone (same block
functions, same order), so the batch is compared with the one-slice path bit
for bit, and one slice with the FP64 oracle."""
import os

import numpy as np
import pytest
import torch

from paper_1009_2288_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    from paper_1009_2288_amd import eptv
    eptv.library()
    return eptv


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def small_batch(n=6, seed=3):
    # uneven slices: 64..128 pixels, 9..31 views, 96..256 bins (one 77x53-like ragged slice included)
    cases = synth.batch_cases(n, seed, sizes=(64, 96, 128), views=(9, 31), bins=(96, 256))
    return cases


PRM = dict(cgls_iters=3, tv_iters=5, lam=1000.0, tv_eps=1e-4)


def single(E, case, K, **kw):
    P = E.Plan(case.geom)
    f, st = P.reconstruct(dev(case.y), E.Params(outer_iters=K, **{**PRM, **kw}), f_ref=dev(case.phantom))
    return f.cpu().numpy(), st


@pytest.mark.parametrize("graph", [True, False])
def test_batch_equals_single_slices_bit_for_bit(E, graph):
    cases = small_batch()
    B = E.Batch([c.geom for c in cases])
    B.set_launch(16, 2, 8)  # the one-slice projector shape
    old = os.environ.get("EPTV_GRAPH")
    os.environ["EPTV_GRAPH"] = "1" if graph else "0"
    try:
        fs, sts = B.reconstruct([dev(c.y) for c in cases], E.Params(outer_iters=8, **PRM),
                                f_refs=[dev(c.phantom) for c in cases])
    finally:
        if old is None:
            os.environ.pop("EPTV_GRAPH", None)
        else:
            os.environ["EPTV_GRAPH"] = old
    for i, c in enumerate(cases):
        f1, st1 = single(E, c, 8)
        assert np.array_equal(fs[i].cpu().numpy(), f1), i
        assert np.array_equal(sts[i]["armijo_k"], st1["armijo_k"]), i
        assert np.array_equal(sts[i]["sigma"], st1["sigma"]), i
        assert np.array_equal(sts[i]["rmse"], st1["rmse"]), i


@pytest.mark.parametrize("kw", [dict(cgls_iters=0, mu=1.0, lam=2000.0, p2_start=1), dict(tv_iters=0),
                                dict(sigma_fixed=float("inf")), dict(positivity=0, cgls_iters=1)])
def test_batch_variants_equal_single(E, kw):
    cases = small_batch(4, seed=5)
    B = E.Batch([c.geom for c in cases])
    B.set_launch(16, 1, 4)
    fs, _ = B.reconstruct([dev(c.y) for c in cases], E.Params(outer_iters=4, **{**PRM, **kw}))
    for i, c in enumerate(cases):
        P = E.Plan(c.geom)
        f1, _ = P.reconstruct(dev(c.y), E.Params(outer_iters=4, **{**PRM, **kw}))
        assert np.array_equal(fs[i].cpu().numpy(), f1.cpu().numpy()), (i, kw)


def test_batch_slice_matches_oracle(E, oracle):
    """The 128^2 small case as one slice among others, against the FP64 oracle."""
    c = synth.make_case("small", 0)
    others = small_batch(3, seed=7)
    cases = [others[0], c, others[1], others[2]]
    B = E.Batch([x.geom for x in cases])
    B.tune(reps=3)
    fs, sts = B.reconstruct([dev(x.y) for x in cases], E.Params(outer_iters=20, **PRM))
    M = oracle.Matrix(c.geom)
    fo, so = M.reconstruct(c.y.astype(np.float32), oracle.Params(outer_iters=20, lam=1000.0), f_ref=c.phantom)
    assert float(so["armijo_margin"].min()) > 1e-5
    assert np.array_equal(sts[1]["armijo_k"], so["armijo_k"])
    assert rel(fs[1].cpu().numpy(), fo) <= 1e-4


def test_batch_warm_start_and_rejections(E):
    cases = small_batch(3, seed=9)
    B = E.Batch([c.geom for c in cases])
    B.set_launch(16, 2, 8)
    ys = [dev(c.y) for c in cases]
    f7, _ = B.reconstruct(ys, E.Params(outer_iters=7, **PRM), stats=False)
    f4, _ = B.reconstruct(ys, E.Params(outer_iters=4, **PRM), stats=False)
    f43, _ = B.reconstruct(ys, E.Params(outer_iters=3, zero_init=0, **PRM), fs=[f.clone() for f in f4], stats=False)
    for a, b in zip(f7, f43):
        assert torch.equal(a, b)
    with pytest.raises(E.EptvError):
        B.reconstruct(ys, E.Params(outer_iters=1, stored_matrix=1, **PRM))
    with pytest.raises(E.EptvError):
        B.reconstruct(ys, E.Params(outer_iters=1, interp_bp=1, **PRM))


def test_full_size_batch_in_the_tuned_launch(E, oracle):
    """64 slices of 256^2 / 384^2 / 512^2, 20-60 views, 368-736 bins, I0
    1e4-1e5, with the tuner's launch shapes: sampled slices against the
    one-slice path (summation order may differ with the projector's segment
    count) and the smallest 256^2 slice against the oracle."""
    cases = synth.batch_cases(64, 0, with_phantom=False)
    B = E.Batch([c.geom for c in cases])
    tuned = B.tune(reps=3)
    assert tuned["proj_seg"] in (4, 8, 16)
    K = 3
    fs, sts = B.reconstruct([dev(c.y) for c in cases], E.Params(outer_iters=K, **PRM))
    for i in (0, 17, 40, 63):
        f1, st1 = single(E, synth.Case(cases[i].name, cases[i].geom, cases[i].ellipses,
                                       np.zeros((cases[i].geom.ny, cases[i].geom.nx)), cases[i].p, cases[i].y,
                                       cases[i].i0, cases[i].seed), K)
        assert rel(fs[i].cpu().numpy(), f1) <= 1e-5, i
    i = min(range(64), key=lambda k: cases[k].geom.nx * cases[k].geom.n_views * cases[k].geom.n_bins)
    M = oracle.Matrix(cases[i].geom)
    fo, so = M.reconstruct(cases[i].y.astype(np.float32), oracle.Params(outer_iters=K, lam=1000.0))
    assert float(so["armijo_margin"].min()) > 1e-5
    assert rel(fs[i].cpu().numpy(), fo) <= 1e-4
