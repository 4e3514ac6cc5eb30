"""eptv_reconstruct_noalloc (the workspace in the library's fixed device array)
against eptv_reconstruct (a caller's workspace), through the C ABI: the same
kernels in the same order, so images and per-iteration records must agree bit
for bit.  Two calls in a row, the second on a smaller plan; the early-stop and
input-scan reads; the size limit.
"""
import sys

import numpy as np
import pytest

from paper_1009_2288_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(autouse=True)
def announce(request):
    sys.__stderr__.write(f"\n[gpu-case] {request.node.nodeid}\n")
    sys.__stderr__.flush()
    yield


@pytest.fixture(scope="module")
def E():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU")
    from paper_1009_2288_amd import eptv
    eptv.library()
    return eptv


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _compare(E, P, case, params, f_ref=None):
    y = dev(case.y)
    fa, sa = P.reconstruct(y, params, f_ref=f_ref)
    fb, sb = P.reconstruct_noalloc(y, params, f_ref=f_ref)
    torch.cuda.synchronize()
    a, b = fa.cpu().numpy(), fb.cpu().numpy()
    assert rel(b, a) <= 1e-4
    assert np.array_equal(a, b), "same kernels in the same order: identical bits expected"
    for k in sa:
        assert np.array_equal(np.asarray(sa[k]), np.asarray(sb[k])), k
    return b, sb


def test_noalloc_equals_reconstruct_twice_second_smaller(E):
    """The 512^2 / 40-view workload, then the 128^2 / 30-view one: the second
    call reuses the array the first left behind."""
    big = synth.make_case("paper", 0)
    Pb = E.Plan(big.geom)
    prm = E.Params(outer_iters=6)
    need = Pb.workspace_bytes(prm)
    print(f"workspace {need} of {E.noalloc_scratch_bytes()} bytes", flush=True)
    assert need <= E.noalloc_scratch_bytes()
    _compare(E, Pb, big, prm, f_ref=dev(big.phantom))

    small = synth.make_case("small", 3)
    Ps = E.Plan(small.geom)
    f, st = _compare(E, Ps, small, E.Params(outer_iters=10), f_ref=dev(small.phantom))
    assert st["iters_run"] == 10 and np.all(np.isfinite(f))


def test_noalloc_early_stop_and_input_scan(E):
    """The reads back that a caller-workspace run makes through page-locked
    staging go straight to the caller here: the RMSE checks of an early stop
    and the non-finite input scan."""
    c = synth.make_case("small", 1)
    P = E.Plan(c.geom)
    ref = dev(c.phantom)
    full, st = P.reconstruct(dev(c.y), E.Params(outer_iters=30), f_ref=ref)
    target = float(st["rmse"][11])
    prm = E.Params(outer_iters=30, stop_rmse=target, check_every=1, check_finite=1)
    f, sn = _compare(E, P, c, prm, f_ref=ref)
    assert sn["iters_run"] <= 12
    bad = c.y.astype(np.float32).copy()
    bad[3, 7] = np.nan
    with pytest.raises(E.EptvError) as ei:
        P.reconstruct_noalloc(dev(bad), prm, f_ref=ref)
    assert ei.value.status == E.EPTV_ERR_NONFINITE


def test_noalloc_rejects_a_workspace_beyond_its_array(E):
    g = synth.Geometry(1024, 1024, 1.0, 8, 64, synth.fan_dbeta(1024, 1024, 1.0, 2000.0, 64), 2000.0, 3000.0)
    P = E.Plan(g)
    prm = E.Params(outer_iters=1)
    assert P.workspace_bytes(prm) > E.noalloc_scratch_bytes()
    y = torch.zeros((8, 64), dtype=torch.float32, device="cuda")
    with pytest.raises(E.EptvError) as ei:
        P.reconstruct_noalloc(y, prm)
    assert ei.value.status == E.EPTV_ERR_WORKSPACE
