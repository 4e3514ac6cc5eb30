"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Both sides receive identical float32-representable inputs (the oracle widens
them to float64).  Per-call bar: relative L2 <= 1e-5 for P, P^T, the P2
direction and the edge weights, and for sigma; after a fixed number of outer
iterations: relative L2 <= 1e-4 on the image.  Inputs are seeded synthetic
phantoms and random arrays of the two workload shapes plus ragged shapes.
"""
import math
import os
import sys

import numpy as np
import pytest

from paper_1009_2288_amd import synth
from paper_1009_2288_amd.synth import Geometry, fan_dbeta

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


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def ragged_geom():
    return Geometry(77, 53, 1.1, 13, 101, fan_dbeta(77, 53, 1.1, 150.0, 101) * 1.05, 150.0, 300.0, 0.3)


def odd_geom():
    # odd bin count (a ray through the isocentre), odd image, views not a multiple of 4
    return Geometry(65, 65, 1.0, 7, 129, fan_dbeta(65, 65, 1.0, 120.0, 129), 120.0, 240.0)


def wide_geom():
    # 1100 pixels wide, two views 45 degrees apart: a 128-entry chunk of a
    # diagonal ray spans more than 65535 image indices, so the stored CSR copy
    # keeps its wide (16-byte slot) encoding
    return Geometry(1100, 1100, 0.5, 2, 64, fan_dbeta(1100, 1100, 0.5, 2000.0, 64), 2000.0, 4000.0,
                    view_angles_rad=np.array([0.0, np.pi / 4]))


GEOMS = {
    "small": synth.geometry_small,
    "paper": synth.geometry_paper,
    "ragged": ragged_geom,
    "odd": odd_geom,
    "wide": wide_geom,
}

_mat_cache = {}


def matrix(oracle, name):
    if name not in _mat_cache:
        _mat_cache[name] = oracle.Matrix(GEOMS[name]())
    return _mat_cache[name]


_plan_cache = {}


def plan(E, name):
    if name not in _plan_cache:
        _plan_cache[name] = E.Plan(GEOMS[name]())
    return _plan_cache[name]


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


# ------------------------------------------------------------------ P and P^T

@pytest.mark.parametrize("name", list(GEOMS))
def test_project_parity(E, oracle, name):
    g = GEOMS[name]()
    M, P = matrix(oracle, name), plan(E, name)
    for seed, img in ((0, synth.random_image(g.nx, g.ny, 1)),
                      (1, synth.raster(synth.phantom_small(3) if g.nx <= 128 else synth.phantom_paper(3), g.nx, g.ny,
                                       g.pixel_mm).astype(np.float32))):
        q = P.project(dev(img)).cpu().numpy()
        assert rel(q, M.project(img)) <= 1e-5, (name, seed)
    # the same kernel fed both layouts by the caller gives the same bits
    img = synth.random_image(g.nx, g.ny, 1)
    qa = P.project(dev(img))
    qb = P.project_dual(dev(img), dev(img.T.copy()))
    assert torch.equal(qa, qb)
    # q = alpha P x + beta q
    x = synth.random_image(g.nx, g.ny, 5)
    q0 = synth.random_sinogram(g.n_views, g.n_bins, 6)
    out = dev(q0)
    P.project(dev(x), out, alpha=-0.5, beta=2.0)
    assert rel(out.cpu().numpy(), -0.5 * M.project(x) + 2.0 * q0) <= 1e-5


@pytest.mark.parametrize("name", list(GEOMS))
def test_backproject_parity(E, oracle, name):
    g = GEOMS[name]()
    M, P = matrix(oracle, name), plan(E, name)
    r = synth.random_sinogram(g.n_views, g.n_bins, 2)
    z = P.backproject(dev(r)).cpu().numpy()
    assert rel(z, M.backproject(r)) <= 1e-5
    r2 = M.project(synth.random_image(g.nx, g.ny, 3)).astype(np.float32)
    z2 = P.backproject(dev(r2)).cpu().numpy()
    assert rel(z2, M.backproject(r2)) <= 1e-5
    z0 = synth.random_image(g.nx, g.ny, 4)
    out = dev(z0)
    P.backproject(dev(r), out, alpha=0.25, beta=-1.0)
    assert rel(out.cpu().numpy(), 0.25 * M.backproject(r) - z0) <= 1e-5


@pytest.mark.parametrize("name", list(GEOMS))
def test_float32_adjoint(E, name):
    """<P x, r> = <x, P^T r> for the float32 operators: they are exact transposes,
    so the two sides differ only by float32 summation."""
    g = GEOMS[name]()
    P = plan(E, name)
    rng = np.random.default_rng(7)
    x = rng.normal(size=(g.ny, g.nx)).astype(np.float32)
    r = rng.normal(size=(g.n_views, g.n_bins)).astype(np.float32)
    px = P.project(dev(x)).cpu().numpy().astype(np.float64)
    ptr = P.backproject(dev(r)).cpu().numpy().astype(np.float64)
    a, b = np.vdot(px, r), np.vdot(x, ptr)
    scale = np.linalg.norm(px) * np.linalg.norm(r)
    assert abs(a - b) <= 1e-6 * scale


@pytest.mark.parametrize("name", list(GEOMS))
def test_nnz_matches_oracle(E, oracle, name):
    M, P = matrix(oracle, name), plan(E, name)
    assert abs(P.nnz - M.nnz) <= 1e-4 * M.nnz


def test_ray_on_grid_line(E, oracle):
    """theta = 0 exactly, odd bin count, even image: the central ray lies on a grid
    line and goes wholly to the row above it on both sides."""
    g = Geometry(16, 16, 1.0, 1, 9, fan_dbeta(16, 16, 1.0, 60.0, 9), 60.0, 120.0, 0.0, np.array([0.0]))
    M, P = oracle.Matrix(g), E.Plan(g)
    x = synth.random_image(16, 16, 11)
    assert rel(P.project(dev(x)).cpu().numpy(), M.project(x)) <= 1e-6
    r = synth.random_sinogram(1, 9, 12)
    assert rel(P.backproject(dev(r)).cpu().numpy(), M.backproject(r)) <= 1e-6


# ------------------------------------------------------------------ TV terms and sigma

@pytest.mark.parametrize("name", ["small", "paper", "ragged"])
def test_tv_gradient_and_weights_parity(E, oracle, name):
    g = GEOMS[name]()
    P = plan(E, name)
    f = synth.random_image(g.nx, g.ny, 21, 0.0, 0.03)
    v = synth.random_image(g.nx, g.ny, 22, 0.0, 0.03)
    for sigma in (0.004, 0.02, float("inf")):
        gg, wx, wy = P.tv_gradient(dev(f), dev(v), 1000.0, sigma, 1e-6)
        go, wxo, wyo = oracle.tv_gradient(f, v, 1000.0, sigma, 1e-6)
        assert rel(gg.cpu().numpy(), go) <= 1e-5, sigma
        assert rel(wx.cpu().numpy(), wxo) <= 1e-5
        assert rel(wy.cpu().numpy(), wyo) <= 1e-5


@pytest.mark.parametrize("name", ["small", "paper", "ragged"])
def test_select_sigma_parity(E, oracle, name):
    g = GEOMS[name]()
    P = plan(E, name)
    f = synth.raster(synth.phantom_small(4), g.nx, g.ny, g.pixel_mm).astype(np.float32)
    f += synth.random_image(g.nx, g.ny, 23, -0.002, 0.002)
    for q in (0.9, 0.95, 0.05, 1.0, 1e-9):
        s = float(P.select_sigma(dev(f), q, 1e-6).cpu()[0])
        so = oracle.select_sigma(f, 1e-6, q, 1e-12)
        assert abs(s - so) <= 1e-5 * so, q


def test_select_sigma_exact_on_rectangle(E):
    """A 3 x 5 rectangle (height 1/64, exact in float32, eps = 0) has a known
    multiset of half-edge magnitudes; every order statistic is exact."""
    g = Geometry(16, 16, 1.0, 4, 32, fan_dbeta(16, 16, 1.0, 60.0, 32), 60.0, 120.0)
    P = E.Plan(g)
    h = 1.0 / 64
    f = np.zeros((16, 16), np.float32)
    f[4:9, 3:6] = h
    r2 = math.sqrt(2.0)
    vals = [h] * (2 * 1 + 2 * 3) + [3 * h / (2 * r2)] * 8 + [h / r2] * (4 * 2 + 4 * 4) + [h / (2 * r2)] * 8
    allv = np.sort(np.array(vals + [0.0] * (2 * 16 * 17 - len(vals))))
    for q in (0.95, 0.97, 0.99, 1.0):
        s = float(P.select_sigma(dev(f), q, 0.0, 1e-30).cpu()[0])
        want = allv[math.ceil(q * allv.size) - 1]
        assert abs(s - want) <= 2e-7 * want, q


def test_tv_step_parity(E, oracle):
    g = GEOMS["small"]()
    P = plan(E, "small")
    c = synth.make_case("small", 0)
    v = c.phantom.astype(np.float32) + synth.random_image(g.nx, g.ny, 31, -0.003, 0.003)
    for sigma in (-1.0, 0.005, float("inf")):
        prm = E.Params(lam=1000.0)
        f = dev(v)
        ks, sg = P.tv_step(f, dev(v), prm, 6, sigma)
        op = oracle.Params(lam=1000.0)
        fo, ko, mo, so = oracle.tv_step(v, v, op, 6, sigma)
        assert list(ks) == list(ko), (sigma, ks, ko, mo)
        assert rel(f.cpu().numpy(), fo) <= 1e-5
        if sigma < 0:
            assert abs(sg - so) <= 1e-5 * so


# ------------------------------------------------------------------ the whole iteration

def oracle_params(oracle, K, **kw):
    return oracle.Params(outer_iters=K, lam=kw.pop("lam", 1000.0), **kw)


def run_pair(E, oracle, name, case, K, **kw):
    P = plan(E, name)
    M = matrix(oracle, name)
    y = case.y.astype(np.float32)
    okw = {k: v for k, v in kw.items() if k != "stored_matrix"}
    fo, so = M.reconstruct(y, oracle_params(oracle, K, **okw), f_ref=case.phantom)
    prm = E.Params(outer_iters=K, lam=kw.pop("lam", 1000.0), **kw)
    f, sg = P.reconstruct(dev(y), prm, f_ref=dev(case.phantom))
    return f.cpu().numpy(), sg, fo, so


def well_separated(so, tol=1e-5):
    """The oracle's own Armijo decisions are far from ties (relative margin >
    tol), so float32 arithmetic cannot flip them; parity of the whole
    trajectory is then expected to the 1e-4 bar."""
    return float(so["armijo_margin"].min()) > tol


def test_reconstruct_small_case(E, oracle):
    """128^2 / 30 views / 256 bins, 50 outer iterations (M = 3, T = 5)."""
    c = synth.make_case("small", 0)
    f, sg, fo, so = run_pair(E, oracle, "small", c, 50)
    assert well_separated(so)
    assert np.array_equal(sg["cgls_steps"], so["cgls_steps"])
    np.testing.assert_allclose(sg["sigma"], so["sigma"], rtol=1e-4)
    assert (sg["armijo_k"] == so["armijo_k"]).mean() >= 0.99, (sg["armijo_k"], so["armijo_k"])
    assert rel(f, fo) <= 1e-4
    np.testing.assert_allclose(sg["rmse"], so["rmse"], rtol=1e-4)
    np.testing.assert_allclose(sg["cgls_resid"], so["cgls_resid"], rtol=1e-4)


def test_reconstruct_paper_case_20_iterations(E, oracle):
    """512^2 / 40 views / 736 bins at the full size, 20 outer iterations."""
    c = synth.make_case("paper", 0)
    f, sg, fo, so = run_pair(E, oracle, "paper", c, 20)
    assert well_separated(so)
    assert np.array_equal(sg["armijo_k"], so["armijo_k"])
    assert rel(f, fo) <= 1e-4
    np.testing.assert_allclose(sg["sigma"], so["sigma"], rtol=1e-4)


@pytest.mark.parametrize("stored", [0, 1, 2], ids=["fly", "stored", "fly_P_stored_PT"])
def test_reconstruct_paper_case_100_iterations_replay(E, oracle, stored):
    """512^2 / 40 x 736 over the workload's full K = 100, in replay mode: the
    GPU runs free and records its Armijo indices; the oracle takes them
    instead of searching and certifies each against its own FP64 inequality
    (slack 1e-6 |Q0|: over these 500 decisions the oracle's own free run has
    two near-ties below 1e-5, where float32 may decide either way), and then
    the images must agree to 1e-4.  With P and P^T on the fly, from the
    stored matrix, and P on the fly with P^T stored."""
    c = synth.make_case("paper", 0)
    P = plan(E, "paper")
    if stored:
        P.store_matrix()
    M = matrix(oracle, "paper")
    y = c.y.astype(np.float32)
    f, sg = P.reconstruct(dev(y), E.Params(outer_iters=100, lam=1000.0, stored_matrix=stored),
                          f_ref=dev(c.phantom))
    fo, so = M.reconstruct(y, oracle_params(oracle, 100), f_ref=c.phantom, armijo_replay=sg["armijo_k"])
    worst = float(so["armijo_margin"].min())
    print("replay certification: min margin", worst, "steps", sg["armijo_k"].size)
    assert worst >= -1e-6
    rs = np.abs(sg["sigma"] - so["sigma"]) / so["sigma"]
    rr = np.abs(sg["rmse"] - so["rmse"]) / so["rmse"]
    print("image", rel(f.cpu().numpy(), fo), "sigma max rel", rs.max(), "at", rs.argmax(), "rmse max rel", rr.max())
    assert rel(f.cpu().numpy(), fo) <= 1e-4
    np.testing.assert_allclose(sg["rmse"], so["rmse"], rtol=1e-4)
    # sigma is an order statistic of neighbour differences (~5e-4 mm^-1) of
    # images whose values (~2e-2) agree to ~1e-5: the same absolute deviation
    # (<= 2 max |f_gpu - f_oracle| per half-edge, the statistic being
    # 1-Lipschitz) is ~40x larger relative to sigma than to the image
    np.testing.assert_allclose(sg["sigma"], so["sigma"], rtol=1e-3)


@pytest.mark.parametrize("kw", [dict(cgls_iters=0, mu=1.0, lam=2000.0, p2_start=1),
                                dict(tv_iters=0), dict(sigma_fixed=float("inf")),
                                dict(cgls_iters=1, tv_iters=2, edge_quantile=0.5, positivity=0)])
def test_reconstruct_variants_ragged(E, oracle, kw):
    g = GEOMS["ragged"]()
    ell = synth.phantom_small(7)
    for e in ell:
        e.cx *= 0.35
        e.cy *= 0.35
        e.a *= 0.35
        e.b *= 0.35
    p = synth.line_integrals(ell, g)
    y = synth.noisy_sinogram(p, 2e4, 99)
    case = synth.Case("ragged", g, ell, synth.raster(ell, g.nx, g.ny, g.pixel_mm), p, y, 2e4, 7)
    f, sg, fo, so = run_pair(E, oracle, "ragged", case, 8, **dict(kw))
    assert rel(f, fo) <= 1e-4, kw


@pytest.mark.parametrize("stored", [0, 1, 2], ids=["fly", "stored", "fly_P_stored_PT"])
def test_reconstruct_is_deterministic_and_graph_equals_direct(E, monkeypatch, stored):
    c = synth.make_case("small", 1)
    P = plan(E, "small")
    if stored:
        P.store_matrix()
    prm = E.Params(outer_iters=6, stored_matrix=stored)
    y = dev(c.y)
    monkeypatch.delenv("EPTV_GRAPH", raising=False)
    f1, _ = P.reconstruct(y, prm, stats=False)
    f2, _ = P.reconstruct(y, prm, stats=False)
    monkeypatch.setenv("EPTV_GRAPH", "1")
    f3, _ = P.reconstruct(y, prm, stats=False)
    f4, _ = P.reconstruct(y, prm, stats=False)  # the captured graph replayed by a second call
    torch.cuda.synchronize()
    assert torch.equal(f1, f2) and torch.equal(f1, f3) and torch.equal(f1, f4)


@pytest.mark.parametrize("every", [0, 2], ids=["no_checks", "checks_every_2"])
def test_stored_iteration_close_folded_equals_own_launch(E, monkeypatch, every):
    """With the stored matrix and direct launches, each outer iteration's close
    (records, counter, state reset) runs in one extra block of the next
    iteration's first projector launch; with a captured graph it is a launch
    of its own.  Both give the same image and the same records bit for bit,
    also when RMSE checks (stop_rmse, never reached here) make the checked
    iterations close in their own launch."""
    c = synth.make_case("small", 1)
    P = plan(E, "small")
    P.store_matrix()
    kw = dict(outer_iters=7, stored_matrix=1)
    if every:
        kw.update(stop_rmse=1e-12, check_every=every)
    prm = E.Params(**kw)
    y, ref = dev(c.y), dev(c.phantom)
    monkeypatch.delenv("EPTV_GRAPH", raising=False)
    f1, s1 = P.reconstruct(y, prm, f_ref=ref)
    monkeypatch.setenv("EPTV_GRAPH", "1")
    f2, s2 = P.reconstruct(y, prm, f_ref=ref)
    torch.cuda.synchronize()
    assert torch.equal(f1, f2)
    assert set(s1) == set(s2)
    for k in s1:
        assert np.array_equal(np.asarray(s1[k]), np.asarray(s2[k])), k
    assert len(s1["rmse"]) == 7 and np.all(np.asarray(s1["rmse"]) > 0)


@pytest.mark.parametrize("name,stored", [("small", 0), ("small", 1), ("ragged", 0), ("odd", 1)])
def test_sigma_from_last_cgls_launch_equals_selection_entry(E, name, stored):
    """The last CGLS step's launch also forms the half-edge histogram of v
    (sigma's first digit, Eq. 5 with sigma as an order statistic of the
    magnitudes): the sigma an outer iteration records equals, bit for bit,
    the selection entry point run on that iteration's v (the same iteration
    with no P2 step and positivity off, whose CGLS launches leave the
    histogram to the selection)."""
    g = GEOMS[name]()
    P = plan(E, name)
    if stored:
        P.store_matrix()
    y = dev(synth.make_case("small", 4).y) if name == "small" else dev(synth.random_image(g.n_bins, g.n_views, 4))
    base = dict(outer_iters=1, stored_matrix=stored)
    v, _ = P.reconstruct(y, E.Params(tv_iters=0, positivity=0, **base), stats=False)
    prm = E.Params(**base)
    _, rec = P.reconstruct(y, prm)
    s_ref = P.select_sigma(v, prm.edge_quantile, prm.tv_eps, prm.sigma_floor)
    torch.cuda.synchronize()
    assert np.float32(rec["sigma"][0]).tobytes() == s_ref.cpu().numpy().astype(np.float32)[0].tobytes()


def test_warm_start_split_equals_straight_run(E):
    """Resume: K1 iterations then K2 more from the result equals K1 + K2 in one call."""
    c = synth.make_case("small", 2)
    P = plan(E, "small")
    y = dev(c.y)
    fa, _ = P.reconstruct(y, E.Params(outer_iters=7), stats=False)
    fb, _ = P.reconstruct(y, E.Params(outer_iters=4), stats=False)
    fb, _ = P.reconstruct(y, E.Params(outer_iters=3, zero_init=0), f=fb, stats=False)
    torch.cuda.synchronize()
    assert torch.equal(fa, fb)


def test_workspace_and_argument_errors(E):
    P = plan(E, "small")
    lib = E.library()
    x = torch.zeros((128, 128), device="cuda")
    q = torch.zeros((30, 256), device="cuda")
    ws = P.workspace()
    need = P.workspace_bytes()
    assert lib.eptv_project(P._h, x.data_ptr(), q.data_ptr(), 1.0, 0.0, ws.data_ptr(), need - 1, None) == 3
    assert lib.eptv_project(P._h, x.data_ptr(), q.data_ptr(), 1.0, 0.0, None, need, None) == 3
    assert lib.eptv_project(P._h, x.data_ptr(), q.data_ptr(), 1.0, 0.0, ws.data_ptr() + 8, need, None) == 3
    with pytest.raises(E.EptvError):
        P.reconstruct(torch.zeros((30, 256), device="cuda"), E.Params(outer_iters=2, cgls_iters=65))
    for sm in (-1, 3):
        with pytest.raises(E.EptvError):
            P.reconstruct(torch.zeros((30, 256), device="cuda"), E.Params(outer_iters=1, stored_matrix=sm))
    fresh = E.Plan(GEOMS["small"]())  # no stored matrix: both stored modes are refused
    for sm in (1, 2):
        with pytest.raises(E.EptvError):
            fresh.reconstruct(torch.zeros((30, 256), device="cuda"), E.Params(outer_iters=1, stored_matrix=sm))
    with pytest.raises(ValueError):
        P.project(torch.zeros((64, 128), device="cuda"))
    with pytest.raises(TypeError):
        P.project(torch.zeros((128, 128), device="cuda", dtype=torch.float64))


def test_zero_iterations_and_empty_steps(E):
    P = plan(E, "small")
    c = synth.make_case("small", 0)
    f0 = dev(c.phantom)
    f, st = P.reconstruct(dev(c.y), E.Params(outer_iters=0, zero_init=0), f=f0.clone())
    assert torch.equal(f, f0)
    f1 = f0.clone()
    ks, _ = P.tv_step(f1, f0, E.Params(), 0, 0.01)
    assert len(ks) == 0 and torch.equal(f1, f0)


# ------------------------------------------------------------------ the stored matrix (Sec. 2.3 look-up tables)

@pytest.mark.parametrize("name", ["small", "paper", "ragged", "odd", "wide"])
def test_stored_matrix_parity(E, oracle, name):
    g = GEOMS[name]()
    M, P = matrix(oracle, name), plan(E, name)
    nbytes = P.store_matrix()
    # compact CSR (6 bytes per entry) + CSC (8), or the wide CSR (8) + CSC (8)
    lay = P.stored_layout()
    assert lay["csr_compact"] == (name != "wide")
    assert lay["csr_bytes"] + lay["csc_bytes"] == nbytes
    assert lay["csc_bytes"] >= 8 * P.nnz and lay["csr_bytes"] >= (6 if lay["csr_compact"] else 8) * P.nnz
    x = synth.random_image(g.nx, g.ny, 41)
    r = synth.random_sinogram(g.n_views, g.n_bins, 42)
    qs = P.project_stored(dev(x)).cpu().numpy()
    zs = P.backproject_stored(dev(r)).cpu().numpy()
    assert rel(qs, M.project(x)) <= 1e-5
    assert rel(zs, M.backproject(r)) <= 1e-5
    # the same float32 matrix as the on-the-fly kernels: only summation order differs
    assert rel(qs, P.project(dev(x)).cpu().numpy()) <= 1e-6
    assert rel(zs, P.backproject(dev(r)).cpu().numpy()) <= 1e-6
    out = dev(q0 := synth.random_sinogram(g.n_views, g.n_bins, 43))
    P.project_stored(dev(x), out, alpha=2.0, beta=-1.0)
    assert rel(out.cpu().numpy(), 2.0 * M.project(x) - q0) <= 1e-5
    # the caller's transposed copy gives the same result bit for bit
    xd = dev(x)
    assert torch.equal(P.project_stored_dual(xd, xd.t().contiguous()), P.project_stored(xd))


@pytest.mark.parametrize("stored", [1, 2], ids=["stored", "fly_P_stored_PT"])
def test_reconstruct_stored_matrix(E, oracle, stored):
    c = synth.make_case("small", 0)
    P = plan(E, "small")
    P.store_matrix()
    f, sg, fo, so = run_pair(E, oracle, "small", c, 50, stored_matrix=stored)
    assert well_separated(so)
    assert np.array_equal(sg["armijo_k"], so["armijo_k"])
    assert rel(f, fo) <= 1e-4


# ------------------------------------------------------------------ Eq. 11 backprojector (App. III)

@pytest.mark.parametrize("name", ["small", "paper", "ragged", "odd"])
def test_backproject_interp_parity(E, oracle, name):
    g = GEOMS[name]()
    P = plan(E, name)
    for seed, r in ((51, synth.random_sinogram(g.n_views, g.n_bins, 51)),
                    (52, synth.make_case("small", 0).p if name == "small" else None)):
        if r is None:
            continue
        z = P.backproject_interp(dev(r)).cpu().numpy()
        assert rel(z, oracle.backproject_interp(g, r)) <= 1e-5, seed
    c0 = synth.random_image(g.nx, g.ny, 53)
    out = dev(c0)
    P.backproject_interp(dev(r := synth.random_sinogram(g.n_views, g.n_bins, 54)), out, alpha=0.5, beta=2.0)
    assert rel(out.cpu().numpy(), 0.5 * oracle.backproject_interp(g, r) + 2.0 * c0) <= 1e-5


@pytest.mark.parametrize("K,kw", [(30, dict()), (5, dict(cgls_iters=0, mu=1.0, lam=2000.0, p2_start=1))])
def test_reconstruct_interp_bp(E, oracle, K, kw):
    """P1 with the Eq. 11 operator in place of P^T.  The gradient form of P1
    with it is far less stable: the oracle's own image moves by 1.4e-6 after
    10 iterations and 4e-5 after 20 for a 6e-8 relative change of y (1e-8
    after 5), so it is compared over 5 iterations."""
    c = synth.make_case("small", 0)
    f, sg, fo, so = run_pair(E, oracle, "small", c, K, interp_bp=1, **kw)
    assert well_separated(so)
    assert np.array_equal(sg["armijo_k"], so["armijo_k"])
    assert rel(f, fo) <= 1e-4


# ------------------------------------------------------------------ given (frozen) edge weights

@pytest.mark.parametrize("frozen", [3, 20])
def test_reconstruct_with_given_weights(E, oracle, frozen):
    """Weights proposed from outside (here: Eq. 5's weights of a blurred phantom)
    used in place of Eq. 5 for the first iterations, then adaptive."""
    c = synth.make_case("small", 0)
    g = c.geom
    P, M = plan(E, "small"), matrix(oracle, "small")
    _, wx, wy = oracle.tv_gradient(c.phantom, c.phantom, 1.0, 0.004, 1e-4)
    wx, wy = wx.astype(np.float32), wy.astype(np.float32)
    y = c.y.astype(np.float32)
    K = 20
    fo, so = M.reconstruct(y, oracle_params(oracle, K), f_ref=c.phantom, weights=(wx, wy), frozen_iters=frozen)
    f, sg = P.reconstruct(dev(y), E.Params(outer_iters=K, lam=1000.0), f_ref=dev(c.phantom),
                          weights=(dev(wx), dev(wy)), frozen_iters=frozen)
    assert well_separated(so)
    assert np.array_equal(sg["armijo_k"], so["armijo_k"])
    assert np.all(sg["sigma"][:frozen] == -1.0)
    assert rel(f.cpu().numpy(), fo) <= 1e-4


def test_early_stop_at_the_rmse_target(E):
    """stop_rmse: the run ends at the first checked iteration whose RMSE record
    is at or below the target, with the image of a run of exactly that many
    iterations; with check_every = 4 only every 4th record is looked at."""
    c = synth.make_case("small", 0)
    P = plan(E, "small")
    y, ref = dev(c.y.astype(np.float32)), dev(c.phantom)
    K = 50
    _, full = P.reconstruct(y, E.Params(outer_iters=K, lam=1000.0), f_ref=ref)
    target = float(np.sort(full["rmse"])[K // 3])
    hit = int(np.nonzero(full["rmse"] <= target)[0][0]) + 1
    f1, s1 = P.reconstruct(y, E.Params(outer_iters=K, lam=1000.0, stop_rmse=target), f_ref=ref)
    assert s1["iters_run"] == hit and hit < K
    f2, _ = P.reconstruct(y, E.Params(outer_iters=hit, lam=1000.0), f_ref=ref)
    assert torch.equal(f1, f2)
    np.testing.assert_array_equal(s1["rmse"], full["rmse"][:hit])
    _, s4 = P.reconstruct(y, E.Params(outer_iters=K, lam=1000.0, stop_rmse=target, check_every=4), f_ref=ref)
    checked = [k for k in range(4, K + 1, 4) if full["rmse"][k - 1] <= target]
    assert s4["iters_run"] == (checked[0] if checked else K)
    # no reference image: nothing to check, the full count runs
    _, s0 = P.reconstruct(y, E.Params(outer_iters=7, lam=1000.0, stop_rmse=target))
    assert s0["iters_run"] == 7


def test_replay_of_recorded_decisions(E):
    """eptv_reconstruct_replay: the recorded decisions reproduce the free run
    bit for bit; a changed decision is taken as given; out-of-range indices
    are rejected."""
    c = synth.make_case("small", 1)
    P = plan(E, "small")
    y = dev(c.y.astype(np.float32))
    prm = E.Params(outer_iters=6, lam=1000.0)
    f1, s1 = P.reconstruct(y, prm)
    f2, s2 = P.reconstruct(y, prm, armijo_replay=s1["armijo_k"])
    assert torch.equal(f1, f2)
    assert np.array_equal(s2["armijo_k"], s1["armijo_k"])
    alt = s1["armijo_k"].copy()
    alt[2, 0] += 1
    f3, s3 = P.reconstruct(y, prm, armijo_replay=alt)
    assert np.array_equal(s3["armijo_k"], alt)
    assert not torch.equal(f3, f1)
    with pytest.raises(E.EptvError):
        P.reconstruct(y, prm, armijo_replay=np.full_like(alt, 21))
