"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check uses a closed form,
an independent brute-force construction, an exact identity or invariant, a
textbook special case or a library routine.  CPU only.
"""
import math

import numpy as np
import pytest

from paper_1009_2288_amd.synth import Geometry, fan_dbeta


def geom(nx, ny, V, B, sad=60.0, pixel=1.0, angles=None, offset=0.0, fan_scale=1.0):
    dbeta = fan_dbeta(nx, ny, pixel, sad, B) * fan_scale
    return Geometry(nx, ny, pixel, V, B, dbeta, sad, 2 * sad, offset,
                    None if angles is None else np.asarray(angles, float))


def rays(g):
    """Source point and unit direction of every ray, written from the scanner
    description (source at -SAD(cos t, sin t), ray along t + beta_b)."""
    th = g.angles()[:, None]
    beta = (np.arange(g.n_bins)[None, :] - 0.5 * (g.n_bins - 1) + g.bin_offset) * g.dbeta_rad
    sx = np.broadcast_to(-g.sad_mm * np.cos(th), (g.n_views, g.n_bins))
    sy = np.broadcast_to(-g.sad_mm * np.sin(th), (g.n_views, g.n_bins))
    return sx, sy, np.cos(th + beta), np.sin(th + beta)


def clip_len(sx, sy, dx, dy, xlo, xhi, ylo, yhi):
    """Length of the line s + a d inside the half-open box [xlo,xhi) x [ylo,yhi)
    by slab clipping (independent of Siddon's sorted-crossing traversal)."""
    amin, amax = -np.inf, np.inf
    for s, d, lo, hi in ((sx, dx, xlo, xhi), (sy, dy, ylo, yhi)):
        if d != 0.0:
            a1, a2 = (lo - s) / d, (hi - s) / d
            amin, amax = np.maximum(amin, np.minimum(a1, a2)), np.minimum(amax, np.maximum(a1, a2))
        else:
            inside = (s >= lo) & (s < hi)
            amax = np.where(inside, amax, -np.inf)
    return np.maximum(amax - amin, 0.0)


def dense_bruteforce(g):
    nx, ny, d = g.nx, g.ny, g.pixel_mm
    xe = (np.arange(nx + 1) - 0.5 * nx) * d
    ye = (np.arange(ny + 1) - 0.5 * ny) * d
    XL, YL = np.meshgrid(xe[:-1], ye[:-1])
    XH, YH = np.meshgrid(xe[1:], ye[1:])
    sx, sy, dx, dy = rays(g)
    A = np.zeros((g.n_views * g.n_bins, nx * ny))
    for v in range(g.n_views):
        for b in range(g.n_bins):
            A[v * g.n_bins + b] = clip_len(sx[v, b], sy[v, b], dx[v, b], dy[v, b], XL, XH, YL, YH).ravel()
    return A


def dense_oracle(O, g):
    M = O.Matrix(g)
    rp, col, val = M.csr()
    A = np.zeros((g.n_views * g.n_bins, g.nx * g.ny))
    for r in range(len(rp) - 1):
        A[r, col[rp[r]:rp[r + 1]]] += val[rp[r]:rp[r + 1]]
    return M, A


# ------------------------------------------------------------------ P, P^T (Sec. 2.1 Eq. 1)

@pytest.mark.parametrize("g", [geom(8, 8, 9, 24), geom(5, 7, 7, 13), geom(9, 9, 8, 31, fan_scale=1.3),
                               geom(6, 9, 5, 11, offset=0.25)])
def test_P_bruteforce_dense(oracle, g):
    """Every entry p_ij = |ray_i cap pixel_j| against independent slab clipping."""
    M, A = dense_oracle(oracle, g)
    B = dense_bruteforce(g)
    assert np.abs(A - B).max() < 1e-12 * g.pixel_mm
    x = np.random.default_rng(1).uniform(size=(g.ny, g.nx))
    r = np.random.default_rng(2).uniform(-1, 1, size=(g.n_views, g.n_bins))
    np.testing.assert_allclose(M.project(x).ravel(), B @ x.ravel(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(M.backproject(r).ravel(), B.T @ r.ravel(), rtol=1e-12, atol=1e-12)


def test_P_ray_on_grid_line_goes_to_upper_pixel(oracle):
    """A ray lying exactly on a grid line (theta = 0, central bin, even ny) is
    given wholly to the pixel row above the line (half-open pixels)."""
    g = geom(8, 8, 1, 9, angles=[0.0])
    pix, ln = oracle.trace_ray(g, 0, 4)
    assert np.all(pix // 8 == 4) and sorted(pix % 8) == list(range(8))
    np.testing.assert_allclose(ln, 1.0, rtol=0, atol=1e-12)
    A = dense_oracle(oracle, g)[1]
    np.testing.assert_allclose(A, dense_bruteforce(g), atol=1e-12)


def trapezoid_chord(t, c, s, d):
    """Chord of a line with unit direction (c, s) through a d x d square whose
    centre lies at signed distance t from it: a trapezoid in t."""
    a, b, h = max(abs(c), abs(s)), min(abs(c), abs(s)), 0.5 * d
    t = np.abs(t)
    if b == 0:
        return np.where(t < h, d / a, 0.0)
    return np.where(t <= h * (a - b), d / a, np.clip((h * (a + b) - t) / (a * b), 0.0, None))


def test_P_single_pixel_closed_form(oracle):
    g = geom(16, 16, 12, 40, sad=80.0)
    M = oracle.Matrix(g)
    sx, sy, dx, dy = rays(g)
    rng = np.random.default_rng(3)
    for _ in range(6):
        i, j = rng.integers(0, 16, size=2)
        e = np.zeros((16, 16))
        e[j, i] = 1.0
        q = M.project(e)
        cx, cy = (i + 0.5 - 8) * g.pixel_mm, (j + 0.5 - 8) * g.pixel_mm
        for v in range(g.n_views):
            for b in range(g.n_bins):
                t = -dy[v, b] * (cx - sx[v, b]) + dx[v, b] * (cy - sy[v, b])
                assert abs(q[v, b] - trapezoid_chord(t, dx[v, b], dy[v, b], g.pixel_mm)) < 1e-12


def test_P_all_ones_image_is_box_chord(oracle):
    g = geom(24, 17, 10, 64, sad=70.0, pixel=0.7)
    M = oracle.Matrix(g)
    q = M.project(np.ones((g.ny, g.nx)))
    sx, sy, dx, dy = rays(g)
    X, Y = 0.5 * g.nx * g.pixel_mm, 0.5 * g.ny * g.pixel_mm
    exp = np.vectorize(lambda a, b, c, d: clip_len(a, b, c, d, -X, X, -Y, Y))(sx, sy, dx, dy)
    np.testing.assert_allclose(q, exp, rtol=1e-12, atol=1e-12)


def test_P_disk_converges_to_closed_form(oracle):
    """Uniform disk: P(raster) -> 2 sqrt(r^2 - p^2), error shrinking ~ linearly in the pixel size."""
    errs = []
    R, fov = 40.0, 128.0
    for n in (32, 64, 128):
        d = fov / n
        g = Geometry(n, n, d, 6, 96, 2 * math.asin(0.5 * fov * math.sqrt(2) / 300.0) / 96, 300.0, 600.0)
        k = 16
        c = (np.arange(n * k) + 0.5) / k * d - 0.5 * fov
        X, Y = np.meshgrid(c, c)
        img = (X * X + Y * Y <= R * R).reshape(n, k, n, k).mean(axis=(1, 3))
        q = oracle.Matrix(g).project(img)
        sx, sy, dx, dy = rays(g)
        p = np.abs(-dy * (0 - sx) + dx * (0 - sy))
        exact = 2 * np.sqrt(np.maximum(R * R - p * p, 0))
        errs.append(np.abs(q - exact).max())
    assert errs[2] < 2.0 * 128 / 128  # a couple of pixel widths at most
    assert errs[0] / errs[2] > 2.5  # roughly linear convergence over 4x refinement


def test_adjoint_identity(oracle):
    g = geom(20, 14, 11, 37, sad=50.0)
    M = oracle.Matrix(g)
    rng = np.random.default_rng(4)
    for _ in range(3):
        x = rng.normal(size=(g.ny, g.nx))
        r = rng.normal(size=(g.n_views, g.n_bins))
        a, b = np.vdot(M.project(x), r), np.vdot(x, M.backproject(r))
        assert abs(a - b) <= 1e-12 * (abs(a) + abs(b))


def test_rotation_by_quarter_turn(oracle):
    """With V % 4 == 0 the scanner maps onto itself under a 90 degree turn:
    P(f')[v] = P(f)[v - V/4] for f'(x, y) = f(y, -x)."""
    g = geom(16, 16, 8, 48, sad=70.0)
    M = oracle.Matrix(g)
    f = np.random.default_rng(5).uniform(size=(16, 16))
    fr = f[::-1, :].T
    np.testing.assert_allclose(M.project(fr), np.roll(M.project(f), 2, axis=0), rtol=1e-11, atol=1e-11)


# ------------------------------------------------------------------ Eq. 11 backprojector (App. III)

@pytest.mark.parametrize("offset,bins", [(0.0, (4,)), (0.5, (3, 4)), (-0.5, (4, 5))])
def test_eq11_centre_pixel_closed_form(oracle, offset, bins):
    """The centre pixel of an odd grid sits on the isocentre: every view sees it
    on the central ray (beta* = 0) at distance SAD, so Eq. 11 reads the bin
    whose centre is at beta = 0 (or the mean of the two around it when the
    detector is shifted by half a bin) and divides by SAD."""
    g = geom(5, 5, 7, 9, pixel=0.7, angles=np.random.default_rng(11).uniform(0, 2 * np.pi, 7), offset=offset)
    y = np.random.default_rng(12).uniform(size=(g.n_views, g.n_bins))
    z = oracle.backproject_interp(g, y)
    expect = g.pixel_mm ** 2 / (g.dbeta_rad * g.sad_mm) * sum(y[:, b].sum() for b in bins) / len(bins)
    assert abs(z[2, 2] - expect) <= 1e-12 * expect


def test_eq11_strip_lies_on_the_traced_ray(oracle):
    """For a sinogram with a single non-zero bin, the pixels that Eq. 11 gives at
    least half their full weight d^2 / (dbeta l) have centres within half a bin
    of that ray, so the ray crosses each of them: they must be a subset of the
    ray's Siddon support (itself pinned by brute force above) and cover a good
    part of it."""
    g = geom(32, 32, 4, 160, angles=[0.3, 1.9, 3.4, 5.0])
    M = oracle.Matrix(g)
    half_diag = 0.5 * g.pixel_mm * math.hypot(g.nx, g.ny)
    assert (g.sad_mm + half_diag) * 0.5 * g.dbeta_rad < 0.5 * g.pixel_mm  # strip narrower than a pixel
    px = (np.arange(g.nx) + 0.5 - 0.5 * g.nx) * g.pixel_mm
    py = (np.arange(g.ny) + 0.5 - 0.5 * g.ny) * g.pixel_mm
    for v, b in [(0, 80), (1, 60), (2, 95), (3, 71)]:
        th = g.angles()[v]
        dist = np.hypot(px[None, :] + g.sad_mm * np.cos(th), py[:, None] + g.sad_mm * np.sin(th))
        y = np.zeros((g.n_views, g.n_bins))
        y[v, b] = 1.0
        strip = oracle.backproject_interp(g, y) * dist * g.dbeta_rad / g.pixel_mm ** 2 >= 0.5
        support = M.backproject(y) > 0.0
        assert strip.any() and not (strip & ~support).any()
        assert strip.sum() >= 0.15 * support.sum()


def test_eq11_adjoint_condition_on_smooth_data(oracle):
    """App. III: the operator is built to satisfy <f, P^T y> = <P f, y> (Eq. A3),
    which the paper reports holds to better than 1 %.  On smooth inputs (a
    rasterised phantom and the exact line integrals of another) the defect is
    second order in the sampling and far smaller."""
    from paper_1009_2288_amd import synth
    c = synth.make_case("small", 0)
    M = oracle.Matrix(c.geom)
    other = synth.Ellipse(10.0, -5.0, 30.0, 18.0, 0.4, 0.02)
    y = synth.line_integrals([other], c.geom)
    a = float(np.vdot(M.project(c.phantom), y))
    b = float(np.vdot(c.phantom, M.backproject_interp(y)))
    assert abs(a - b) <= 2e-4 * abs(a)


def test_eq11_scale_matches_transpose_of_constant(oracle):
    """Per view the chords of the rays through a pixel sum to its area over the
    ray spacing l * dbeta, the constant Eq. 11 carries: on a constant sinogram
    the two operators agree when averaged over 8x8 blocks."""
    from paper_1009_2288_amd import synth
    g = synth.geometry_small()
    M = oracle.Matrix(g)
    one = np.ones((g.n_views, g.n_bins))
    k = 8
    blk = lambda z: z.reshape(g.ny // k, k, g.nx // k, k).mean(axis=(1, 3))
    r = blk(M.backproject(one)) / blk(oracle.backproject_interp(g, one))
    c = r[4:12, 4:12]
    assert np.abs(c - 1.0).max() <= 1e-2


def test_eq11_zero_beyond_the_detector(oracle):
    """A pixel seen outside the fan reads nothing (zero beyond the last bin),
    and no view reads a neighbouring view's bins: with a narrow fan, a
    sinogram whose only non-zero bins are the edge bins of the other view gives
    the same image as that view alone."""
    g = geom(9, 9, 1, 5, angles=[0.0], fan_scale=0.2)
    z = oracle.backproject_interp(g, np.ones((1, 5)))
    assert z[4, 4] > 0 and z[0, 4] == 0.0 and z[8, 4] == 0.0
    angles = [0.0, 2.0]
    g2 = geom(9, 9, 2, 5, angles=angles, fan_scale=0.2)
    for keep in (0, 1):
        g1 = geom(9, 9, 1, 5, angles=[angles[keep]], fan_scale=0.2)
        y = np.zeros((2, 5))
        y[keep, 0] = y[keep, 4] = 1.0
        z2 = oracle.backproject_interp(g2, y)
        assert np.array_equal(z2, oracle.backproject_interp(g1, y[keep:keep + 1]))
        assert z2.max() > 0


def test_eq11_in_p1_wiring(oracle):
    """With interp_bp the P1 step uses Eq. 11 in place of P^T: one gradient-form
    step is f - mu/lambda B(P f - y), one CGLS step is u + a s with s = B r,
    a = |s|^2 / |P s|^2 (App. I with B for P^T), B the Eq. 11 operator."""
    g = geom(12, 10, 9, 40)
    M = oracle.Matrix(g)
    rng = np.random.default_rng(21)
    f0 = rng.uniform(size=(g.ny, g.nx))
    y = M.project(rng.uniform(size=(g.ny, g.nx)))
    base = dict(outer_iters=1, tv_iters=0, zero_init=0, positivity=0, interp_bp=1, sigma_fixed=1.0)
    mu, lam = 1.0, 50.0
    f, _ = M.reconstruct(y, oracle.Params(cgls_iters=0, mu=mu, lam=lam, **base), f0=f0)
    np.testing.assert_allclose(f, f0 - mu / lam * M.backproject_interp(M.project(f0) - y), rtol=1e-12, atol=1e-12)
    f, _ = M.reconstruct(y, oracle.Params(cgls_iters=1, **base), f0=f0)
    s = M.backproject_interp(y - M.project(f0))
    a = np.vdot(s, s) / np.vdot(M.project(s), M.project(s))
    np.testing.assert_allclose(f, f0 + a * s, rtol=1e-12, atol=1e-12)


def test_nnz_small_case(oracle):
    """Every ray of the 128^2 case crosses the image; each meets between max(n)
    and nx+ny-1 pixels."""
    from paper_1009_2288_amd.synth import geometry_small
    g = geometry_small()
    M = oracle.Matrix(g)
    rp, _, _ = M.csr()
    cnt = np.diff(rp)
    assert cnt.max() <= g.nx + g.ny - 1
    assert M.nnz == cnt.sum()


# ------------------------------------------------------------------ TV terms (App. II)

def rect_image(n, a, b, h, i0=3, j0=4):
    f = np.zeros((n, n))
    f[j0:j0 + b, i0:i0 + a] = h
    return f


def rect_edge_multiset(a, b, h):
    """Nonzero half-edge magnitudes of an a x b rectangle of height h (eps = 0),
    worked out from Eq. A3 by hand: (value, count)."""
    r2 = math.sqrt(2.0)
    return [(h, 2 * (a - 2) + 2 * (b - 2)), (3 * h / (2 * r2), 8), (h / r2, 4 * (a - 1) + 4 * (b - 1)),
            (h / (2 * r2), 8)]


@pytest.mark.parametrize("a,b,h", [(2, 2, 1.0), (3, 5, 0.02), (7, 4, 2.5)])
def test_tv_rectangle_closed_form(oracle, a, b, h):
    f = rect_image(16, a, b, h)
    J = oracle.tv_energy(f, float("inf"), 0.0)
    closed = h * ((2 + 2 * math.sqrt(2)) * (a + b) + 4 * math.sqrt(2) - 8)
    assert abs(J - closed) < 1e-13 * closed
    tvx, tvy = oracle.tv_edges(f, 0.0)
    vals = np.sort(np.concatenate([tvx.ravel(), tvy.ravel()]))
    exp = []
    for v, c in rect_edge_multiset(a, b, h):
        exp += [v] * c
    exp = np.sort(np.array(exp))
    nz = vals[vals > 0]
    np.testing.assert_allclose(nz, exp, rtol=1e-14)
    # Eq. 5 weights: J = sum count * t exp(-t^2/sigma^2)
    sigma = 0.7 * h
    Jw = oracle.tv_energy(f, sigma, 0.0)
    closed_w = sum(c * v * math.exp(-(v / sigma) ** 2) for v, c in rect_edge_multiset(a, b, h))
    assert abs(Jw - closed_w) < 1e-13 * closed_w
    # sigma as an order statistic of the known multiset (zeros included)
    n = vals.size
    q = 0.995
    assert n == 2 * 16 * 17
    assert oracle.select_sigma(f, 0.0, q, 1e-300) == np.sort(vals)[math.ceil(q * n) - 1]


def test_tv_gradient_rectangle_by_hand(oracle):
    """A2 at hand-computed pixels of a 4 x 3 rectangle of height h (w = 1):
    bottom-left corner 4 sqrt(2)/3, mid left side 1, the pixel left of the
    corner -2 sqrt(2)/3 - sqrt(2) (one flux out of the corner, one from below),
    interior 0."""
    h = 1.0
    f = rect_image(12, 4, 3, h, i0=4, j0=4)
    g, wx, wy = oracle.tv_gradient(f, f, 1.0, float("inf"), 1e-12)
    assert np.all(wx == 1) and np.all(wy == 1)
    r2 = math.sqrt(2.0)
    assert abs(g[4, 4] - 4 * r2 / 3) < 1e-9          # corner (i0, j0)
    assert abs(g[5, 4] - 1.0) < 1e-9                  # left side, middle row
    assert abs(g[5, 5] - 0.0) < 1e-9                  # interior
    # outside neighbour left of the corner: flux h/TV(3h/(2 sqrt 2)) in, transverse edges
    # below it have zero main difference.
    assert abs(g[4, 3] - (-2 * r2 / 3)) < 1e-9


def test_tv_gradient_1d_reduces_to_1d_tv_derivative(oracle):
    """Rows 1..ny-2 of an image constant along y: the y fluxes vanish and A2 is the
    exact derivative of the 1-D weighted TV sum_e w_e sqrt(dh_e^2 + eps^2), w frozen."""
    rng = np.random.default_rng(6)
    nx, ny, eps, sigma, lam = 20, 9, 1e-3, 0.5, 0.3
    h = rng.uniform(0, 1, size=nx)
    f = np.tile(h, (ny, 1))
    v = rng.uniform(0, 1, size=(ny, nx))
    g, wx, _ = oracle.tv_gradient(f, v, lam, sigma, eps)
    hp = np.concatenate([[0.0], h, [0.0]])
    w = np.exp(-(np.diff(hp) ** 2 + eps * eps) / sigma ** 2)  # x-edge weights on an interior row

    def tv1(hh):
        d = np.diff(np.concatenate([[0.0], hh, [0.0]]))
        return np.sum(w * np.sqrt(d * d + eps * eps))

    fd = np.zeros(nx)
    for i in range(nx):
        e = np.zeros(nx)
        e[i] = 1e-6
        fd[i] = (tv1(h + e) - tv1(h - e)) / 2e-6
    for j in range(1, ny - 1):
        np.testing.assert_allclose(g[j] - lam * (f[j] - v[j]), fd, rtol=1e-6, atol=1e-8)
        np.testing.assert_allclose(wx[j], w, rtol=1e-14)


def test_tv_gradient_transpose_symmetry(oracle):
    rng = np.random.default_rng(7)
    f = rng.uniform(size=(11, 13))
    v = rng.uniform(size=(11, 13))
    g, _, _ = oracle.tv_gradient(f, v, 0.7, 0.3, 1e-3)
    gt, _, _ = oracle.tv_gradient(f.T.copy(), v.T.copy(), 0.7, 0.3, 1e-3)
    np.testing.assert_allclose(gt, g.T, rtol=1e-13, atol=1e-14)


def test_tv_gradient_divergence_sums_to_zero(oracle):
    """Discrete divergence theorem: with f zero on a 2-pixel border the A2 term
    telescopes to zero over the image."""
    rng = np.random.default_rng(8)
    f = np.zeros((14, 12))
    f[2:-2, 2:-2] = rng.uniform(size=(10, 8))
    g, _, _ = oracle.tv_gradient(f, f, 1.0, 0.4, 1e-4)
    assert abs(g.sum()) < 1e-12 * np.abs(g).sum()


@pytest.mark.parametrize("sigma", [0.3, np.inf])
def test_tv_vjp_matches_finite_difference_jacobian(oracle, sigma):
    """(dg/df)^T against the Jacobian of the direction g built column by column
    from central differences of g itself (independent of the VJP's formulas)."""
    nx, ny, lam, eps, h = 5, 4, 0.7, 0.05, 1e-6
    rng = np.random.default_rng(31)
    f = rng.normal(size=(ny, nx))
    v = rng.normal(size=(ny, nx))
    n = nx * ny
    J = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = h
        gp = oracle.tv_gradient(f + e.reshape(ny, nx), v, lam, sigma, eps)[0]
        gm = oracle.tv_gradient(f - e.reshape(ny, nx), v, lam, sigma, eps)[0]
        J[:, k] = (gp - gm).ravel() / (2 * h)
    for k in range(3):
        u = rng.normal(size=(ny, nx))
        got = oracle.tv_gradient_vjp(f, u, lam, sigma, eps).ravel()
        np.testing.assert_allclose(got, J.T @ u.ravel(), rtol=1e-6, atol=1e-6 * np.abs(J).max())


def test_tv_vjp_large_eps_is_dirichlet_laplacian(oracle):
    """With sigma = inf and eps far above every difference, F = d / eps and the
    Jacobian tends to lambda I + L / eps, L the 5-point negative Laplacian with
    zero values outside the image."""
    nx, ny, lam, eps = 7, 6, 0.3, 1e5
    rng = np.random.default_rng(32)
    f = rng.uniform(size=(ny, nx))
    u = rng.normal(size=(ny, nx))
    up = np.pad(u, 1)
    lap = 4 * u - up[1:-1, 2:] - up[1:-1, :-2] - up[2:, 1:-1] - up[:-2, 1:-1]
    got = oracle.tv_gradient_vjp(f, u, lam, np.inf, eps)
    np.testing.assert_allclose(got, lam * u + lap / eps, rtol=1e-8, atol=1e-12)


def test_sigma_matches_numpy_inverted_cdf(oracle):
    rng = np.random.default_rng(9)
    f = rng.uniform(0, 0.03, size=(23, 19))
    tvx, tvy = oracle.tv_edges(f, 1e-6)
    allv = np.concatenate([tvx.ravel(), tvy.ravel()])
    for q in (0.05, 0.5, 0.9, 0.95, 1.0):
        assert oracle.select_sigma(f, 1e-6, q, 1e-12) == np.quantile(allv, q, method="inverted_cdf")


def test_sigma_floor_and_infinite_sigma(oracle):
    z = np.zeros((6, 6))
    assert oracle.select_sigma(z, 0.0, 0.9, 1e-12) == 1e-12
    f = np.random.default_rng(10).uniform(size=(6, 6))
    _, wx, wy = oracle.tv_gradient(f, f, 1.0, float("inf"), 1e-6)
    assert np.all(wx == 1.0) and np.all(wy == 1.0)


# ------------------------------------------------------------------ P1: CGLS (App. I)

def full_rank_case(oracle):
    g = geom(8, 8, 12, 24, sad=40.0)
    M, A = dense_oracle(oracle, g)
    assert np.linalg.matrix_rank(A) == 64
    y = np.random.default_rng(11).uniform(0, 1, size=(g.n_views, g.n_bins))
    return g, M, A, y


def test_cgls_reaches_least_squares(oracle):
    g, M, A, y = full_rank_case(oracle)
    u, steps, res = M.cgls(y, np.zeros((8, 8)), 80)
    ls = np.linalg.lstsq(A, y.ravel(), rcond=None)[0]
    cond = np.linalg.cond(A)
    assert np.abs(u.ravel() - ls).max() < 1e-8 * cond * np.abs(ls).max()
    assert abs(res - np.sum((A @ ls - y.ravel()) ** 2)) < 1e-8 * res


def test_cgls_residual_is_non_increasing(oracle):
    g, M, A, y = full_rank_case(oracle)
    u0 = np.random.default_rng(12).uniform(size=(8, 8))
    prev = np.inf
    for m in range(0, 12):
        _, _, res = M.cgls(y, u0, m)
        assert res <= prev * (1 + 1e-12)
        prev = res


# ------------------------------------------------------------------ P2 and the outer loop

def test_armijo_steps_decrease_frozen_surrogate(oracle):
    rng = np.random.default_rng(13)
    v = rng.uniform(0, 0.03, size=(24, 20))
    f = v + rng.normal(0, 0.002, size=v.shape)
    p = oracle.Params(lam=50.0, tv_eps=1e-5)
    for s in range(4):
        g, wx, wy = oracle.tv_gradient(f, v, p.lam, 0.01, p.tv_eps)
        q0 = oracle.surrogate(f, v, p.lam, wx, wy, p.tv_eps)
        f1, ks, _, _ = oracle.tv_step(f, v, p, 1, sigma=0.01)
        assert ks[0] >= 0
        t = (1.0 / p.lam) * 0.5 ** ks[0]
        np.testing.assert_allclose(f1, f - t * g, rtol=1e-14, atol=1e-17)
        q1 = oracle.surrogate(f1, v, p.lam, wx, wy, p.tv_eps)
        assert q1 <= q0 - p.armijo_c * t * np.sum(g * g)
        if ks[0] > 0:  # the previous candidate was rightly rejected
            tp = 2 * t
            qp = oracle.surrogate(f - tp * g, v, p.lam, wx, wy, p.tv_eps)
            assert qp > q0 - p.armijo_c * tp * np.sum(g * g)
        f = f1


def a3_edges_by_definition(f, eps):
    """Every half-edge magnitude of Eq. A3 written out from the equation, one
    edge at a time, with ghost pixels 0 (zero boundary): x-edges [ny][nx+1]
    (entry [j][i+1] = edge (i+1/2, j)), y-edges [ny+1][nx] (entry [j+1][i] =
    edge (i, j+1/2))."""
    ny, nx = f.shape

    def at(i, j):
        return float(f[j, i]) if 0 <= i < nx and 0 <= j < ny else 0.0

    tx = np.zeros((ny, nx + 1))
    ty = np.zeros((ny + 1, nx))
    for j in range(ny):
        for i in range(-1, nx):
            mid = [(at(i, jj) + at(i + 1, jj)) / 2 for jj in (j - 1, j, j + 1)]
            tx[j, i + 1] = math.sqrt((at(i + 1, j) - at(i, j)) ** 2 + (mid[2] - mid[1]) ** 2 / 2
                                     + (mid[1] - mid[0]) ** 2 / 2 + eps * eps)
    for j in range(-1, ny):
        for i in range(nx):
            mid = [(at(ii, j) + at(ii, j + 1)) / 2 for ii in (i - 1, i, i + 1)]
            ty[j + 1, i] = math.sqrt((at(i, j + 1) - at(i, j)) ** 2 + (mid[2] - mid[1]) ** 2 / 2
                                     + (mid[1] - mid[0]) ** 2 / 2 + eps * eps)
    return tx, ty


@pytest.mark.parametrize("a,b,h,lam", [(2, 2, 1.0, 3.0), (3, 5, 0.02, 1000.0), (7, 4, 2.5, 0.25)])
def test_surrogate_rectangle_closed_form(oracle, a, b, h, lam):
    """The P2 energy compared by the Armijo rule (Sec. 2.2 with Eq. 8's
    splitting term; App. II Eq. A3), Q(h) = lambda/2 ||h - v||^2 + sum_e w_e
    TV_e(h), for an a x b rectangle of height h, v = 0, w = 1, eps = 0:
    lambda/2 a b h^2 + h[(2 + 2 sqrt 2)(a + b) + 4 sqrt 2 - 8]."""
    f = rect_image(16, a, b, h)
    ones_x, ones_y = np.ones((16, 17)), np.ones((17, 16))
    q = oracle.surrogate(f, np.zeros_like(f), lam, ones_x, ones_y, 0.0)
    closed = 0.5 * lam * a * b * h * h + h * ((2 + 2 * math.sqrt(2)) * (a + b) + 4 * math.sqrt(2) - 8)
    assert abs(q - closed) <= 1e-13 * closed
    # the data term alone (w = 0): lambda/2, not lambda, times the squared distance to v
    v = np.full_like(f, 0.5 * h)
    q0 = oracle.surrogate(f, v, lam, np.zeros((16, 17)), np.zeros((17, 16)), 0.0)
    assert abs(q0 - 0.5 * lam * (a * b * (0.5 * h) ** 2 + (256 - a * b) * (0.5 * h) ** 2)) <= 1e-13 * q0
    # only the y-edges weighted: their share of the rectangle's multiset, by
    # hand.  The 2a y-edges crossing the top and bottom sides have main
    # difference h (magnitude h, or 3h/(2 sqrt 2) in the 4 corner columns);
    # along each vertical side the columns just inside and just outside hold
    # b - 1 y-edges each with a transverse difference h (h/sqrt 2); the 4
    # y-edges diagonal to the corners see h/2 (h/(2 sqrt 2)).
    qy = oracle.surrogate(f, np.zeros_like(f), lam, np.zeros((16, 17)), ones_y, 0.0)
    r2 = math.sqrt(2.0)
    want_y = h * (2 * (a - 2) + 4 * 3 / (2 * r2) + 4 * (b - 1) / r2 + 4 / (2 * r2))
    assert abs((qy - 0.5 * lam * a * b * h * h) - want_y) <= 1e-13 * want_y


def test_surrogate_with_random_weights_against_eq_a3_by_definition(oracle):
    """Q with independent random weights on the two edge families and a random
    v, against the definition evaluated edge by edge in this test.  That
    evaluation is first tied to the hand-derived half-edge multiset of a
    rectangle, so it is not the oracle's formula retyped unchecked."""
    a, b, h = 4, 3, 0.7
    f = rect_image(12, a, b, h, i0=4, j0=4)
    tx, ty = a3_edges_by_definition(f, 0.0)
    vals = np.sort(np.concatenate([tx.ravel(), ty.ravel()]))
    exp = []
    for val, c in rect_edge_multiset(a, b, h):
        exp += [val] * c
    np.testing.assert_allclose(vals[vals > 0], np.sort(exp), rtol=1e-14)
    rng = np.random.default_rng(41)
    for img, eps in ((f, 0.0), (rng.uniform(0, 0.03, size=(9, 11)), 1e-3)):
        ny, nx = img.shape
        v = rng.uniform(0, 0.03, size=img.shape)
        wx = rng.uniform(0, 1, size=(ny, nx + 1))
        wy = rng.uniform(0, 2, size=(ny + 1, nx))
        lam = 37.0
        tx, ty = a3_edges_by_definition(img, eps)
        want = 0.5 * lam * float(np.sum((img - v) ** 2)) + float(np.sum(wx * tx)) + float(np.sum(wy * ty))
        got = oracle.surrogate(img, v, lam, wx, wy, eps)
        assert abs(got - want) <= 1e-13 * abs(want)
        # each family's weights enter with their own edges (swapped families differ)
        if nx != ny:
            continue
        swapped = oracle.surrogate(img, v, lam, wy.T.copy(), wx.T.copy(), eps)
        assert abs(swapped - got) > 1e-6 * abs(got)


def test_iteration_records_against_direct_computation(oracle):
    """The per-step records of one outer iteration, recomputed independently:
    CGLS gamma_m = ||A^T r_m||^2 and delta_m = ||A s_m||^2 by the App. I
    recurrences written here with the brute-force dense matrix (A f = 0 at the
    zero start), and the Armijo energies Q0 / Q1 of the first descent step as
    the P2 energy evaluated at v and at v - t g with Eq. A3 by definition and
    Eq. 5's weights at v."""
    g, M, A, y = full_rank_case(oracle)
    A = dense_bruteforce(g)
    Mst, lam, eps = 3, 50.0, 1e-3
    p = oracle.Params(outer_iters=1, cgls_iters=Mst, tv_iters=2, lam=lam, tv_eps=eps, sigma_fixed=0.05)
    _, st = M.reconstruct(y, p)
    yv = y.ravel()
    r = yv.copy()
    u = np.zeros(64)
    s = A.T @ r
    gam = s @ s
    for m in range(Mst):
        assert abs(st["cgls_gamma"][0, m] - gam) <= 1e-9 * gam
        q = A @ s
        dl = q @ q
        assert abs(st["cgls_delta"][0, m] - dl) <= 1e-9 * dl
        a = gam / dl
        u += a * s
        r -= a * q
        z = A.T @ r
        gn = z @ z
        s = z + (gn / gam) * s
        gam = gn
    v = u.reshape(8, 8)
    tx, ty = a3_edges_by_definition(v, eps)
    wx, wy = np.exp(-(tx / 0.05) ** 2), np.exp(-(ty / 0.05) ** 2)
    q0 = float(np.sum(wx * tx) + np.sum(wy * ty))  # h = v: no data term
    assert abs(st["armijo_q0"][0, 0] - q0) <= 1e-8 * q0
    k = int(st["armijo_k"][0, 0])
    assert k >= 0
    gdir, _, _ = oracle.tv_gradient(v, v, lam, 0.05, eps)
    h = v - (1.0 / lam) * 0.5 ** k * gdir
    th, tyh = a3_edges_by_definition(h, eps)
    q1 = 0.5 * lam * float(np.sum((h - v) ** 2)) + float(np.sum(wx * th) + np.sum(wy * tyh))
    assert abs(st["armijo_q1"][0, 0] - q1) <= 1e-8 * q1
    assert st["armijo_q1"][0, 0] <= q0


def test_energy_monotone_theorem_case(oracle):
    """Gradient-form P1 with step 1/lambda, lambda >= mu ||P||^2, plain TV
    weights, P2 from f^(k), no truncation: majorisation-minimisation makes
    E = mu/2 ||P f - y||^2 + J_h(f) non-increasing."""
    g, M, A, y = full_rank_case(oracle)
    mu = 1.0
    L = np.linalg.norm(A, 2) ** 2
    p = oracle.Params(outer_iters=25, cgls_iters=0, tv_iters=3, mu=mu, lam=1.01 * mu * L,
                      sigma_fixed=float("inf"), tv_eps=1e-3, p2_start=1, positivity=0, track_energy=1)
    f, st = M.reconstruct(y, p)
    E = st["energy"]
    x0 = 0.5 * mu * np.sum(y ** 2)  # E(f^(0) = 0): J_h(0) = eps * n_edges
    x0 += 1e-3 * 2 * 8 * 9
    E = np.concatenate([[x0], E])
    assert np.all(np.diff(E) <= 1e-12 * np.abs(E[:-1]))
    # independent recomputation of the data term from the brute-force matrix
    dense = dense_bruteforce(g)
    assert abs(0.5 * mu * np.sum((dense @ f.ravel() - y.ravel()) ** 2)
               + oracle.tv_energy(f, float("inf"), 1e-3) - st["energy"][-1]) < 1e-10 * st["energy"][-1]


def test_no_p2_reduces_to_restarted_cgls_least_squares(oracle):
    """With no P2 steps and no truncation the outer loop is restarted CGLS,
    which converges to the least-squares solution on a full-rank system."""
    g, M, A, y = full_rank_case(oracle)
    p = oracle.Params(outer_iters=400, cgls_iters=8, tv_iters=0, positivity=0)
    f, st = M.reconstruct(y, p)
    ls = np.linalg.lstsq(A, y.ravel(), rcond=None)[0]
    assert np.abs(f.ravel() - ls).max() < 1e-6 * np.abs(ls).max()


def test_positivity_truncation(oracle):
    g, M, A, y = full_rank_case(oracle)
    p = oracle.Params(outer_iters=3, cgls_iters=3, tv_iters=2, lam=10.0, positivity=1)
    yy = y - 0.5
    f, _ = M.reconstruct(yy, p)
    assert f.min() >= 0.0
    p.positivity = 0
    f2, _ = M.reconstruct(yy, p)
    assert f2.min() < 0.0


# ------------------------------------------------------------------ the input generator

def test_generator_ellipse_chord_vs_quadrature():
    from paper_1009_2288_amd import synth
    g = geom(16, 16, 3, 7, sad=100.0)
    e = synth.Ellipse(2.0, -1.5, 5.0, 3.0, 0.4, 0.02)
    p = synth.line_integrals([e], g)
    sx, sy, dx, dy = rays(g)
    l = np.linspace(80, 120, 400001)
    for v in range(3):
        for b in range(7):
            X, Y = sx[v, b] + l * dx[v, b], sy[v, b] + l * dy[v, b]
            inside = synth._inside(e, X, Y)
            assert abs(p[v, b] - 0.02 * inside.sum() * (l[1] - l[0])) < 2e-6


def test_generator_poisson_statistics():
    from paper_1009_2288_amd import synth
    p = np.full((200, 500), 1.2)
    y = synth.noisy_sinogram(p, 1e4, 3)
    counts = 1e4 * np.exp(-y)
    lam = 1e4 * math.exp(-1.2)
    n = counts.size
    assert abs(counts.mean() - lam) < 4 * math.sqrt(lam / n)
    assert abs(counts.var() / lam - 1) < 4 * math.sqrt(2.0 / n)


# ------------------------------------------------------------------ given (frozen) edge weights

def _pin_case(oracle):
    g = geom(14, 12, 10, 40)
    M = oracle.Matrix(g)
    rng = np.random.default_rng(41)
    f_true = np.zeros((g.ny, g.nx))
    f_true[3:9, 4:10] = 0.02
    y = M.project(f_true) + 1e-4 * rng.normal(size=(g.n_views, g.n_bins))
    return g, M, y


def test_frozen_unit_weights_are_plain_tv(oracle):
    """w = 1 on every half-edge is Eq. 5 with sigma = inf: plain TV."""
    g, M, y = _pin_case(oracle)
    ones = (np.ones((g.ny, g.nx + 1)), np.ones((g.ny + 1, g.nx)))
    K = 4
    fw, sw = M.reconstruct(y, oracle.Params(outer_iters=K, lam=200.0), weights=ones, frozen_iters=K)
    ft, st = M.reconstruct(y, oracle.Params(outer_iters=K, lam=200.0, sigma_fixed=float("inf")))
    np.testing.assert_array_equal(fw, ft)
    np.testing.assert_array_equal(sw["armijo_k"], st["armijo_k"])


def test_frozen_zero_weights_remove_p2(oracle):
    """w = 0: the direction is lambda (f - v), zero at the start v, so P2 keeps v
    and the iteration is the one without P2."""
    g, M, y = _pin_case(oracle)
    zeros = (np.zeros((g.ny, g.nx + 1)), np.zeros((g.ny + 1, g.nx)))
    fw, _ = M.reconstruct(y, oracle.Params(outer_iters=3, lam=200.0), weights=zeros, frozen_iters=3)
    fn, _ = M.reconstruct(y, oracle.Params(outer_iters=3, lam=200.0, tv_iters=0))
    np.testing.assert_allclose(fw, fn, rtol=0, atol=1e-15)


def test_frozen_then_adaptive(oracle):
    """After the frozen iterations the weights are Eq. 5's again: a run frozen
    for 2 of 5 iterations equals 2 frozen iterations then 3 adaptive ones."""
    g, M, y = _pin_case(oracle)
    rng = np.random.default_rng(42)
    w = (rng.uniform(size=(g.ny, g.nx + 1)), rng.uniform(size=(g.ny + 1, g.nx)))
    f5, s5 = M.reconstruct(y, oracle.Params(outer_iters=5, lam=200.0), weights=w, frozen_iters=2)
    f2, s2 = M.reconstruct(y, oracle.Params(outer_iters=2, lam=200.0), weights=w, frozen_iters=2)
    f3, s3 = M.reconstruct(y, oracle.Params(outer_iters=3, lam=200.0, zero_init=0), f0=f2)
    np.testing.assert_array_equal(f5, f3)
    assert np.all(s5["sigma"][:2] == -1.0) and np.all(s5["sigma"][2:] > 0.0)


# ------------------------------------------------------------------ replay mode

def test_replay_of_own_decisions_reproduces_the_free_run(oracle):
    """Replaying the oracle's own Armijo indices gives the free run's image
    bit for bit, and every decision certifies (margin >= 0: the search would
    make it)."""
    g, M, y = _pin_case(oracle)
    prm = oracle.Params(outer_iters=6, lam=200.0)
    f, st = M.reconstruct(y, prm)
    fr, sr = M.reconstruct(y, prm, armijo_replay=st["armijo_k"])
    np.testing.assert_array_equal(fr, f)
    np.testing.assert_array_equal(sr["armijo_k"], st["armijo_k"])
    assert float(sr["armijo_margin"].min()) >= 0.0
    # for decisions the search agrees with, the signed certification is the
    # search's own decision margin (the same trials, the same distances)
    np.testing.assert_array_equal(sr["armijo_margin"], st["armijo_margin"])


def test_replay_flags_a_wrong_decision(oracle):
    """A replayed index one larger than the search's (a step the search would
    have accepted earlier) and one smaller (a step that fails the rule) both
    certify negative at that step."""
    g, M, y = _pin_case(oracle)
    prm = oracle.Params(outer_iters=3, lam=200.0)
    _, st = M.reconstruct(y, prm)
    ks = st["armijo_k"].copy()
    s = np.argwhere(ks >= 1)[0]
    later = ks.copy()
    later[tuple(s)] += 1
    _, sl = M.reconstruct(y, prm, armijo_replay=later)
    assert sl["armijo_margin"][tuple(s)] < 0.0
    assert np.all(sl["armijo_margin"].reshape(-1)[:np.ravel_multi_index(tuple(s), ks.shape)] >= 0.0)
    earlier = ks.copy()
    earlier[tuple(s)] -= 1
    _, se = M.reconstruct(y, prm, armijo_replay=earlier)
    assert se["armijo_margin"][tuple(s)] < 0.0
