"""Seeded synthetic inputs for the EPTV fan-beam reconstruction path.

This module produces the *inputs* of the method: scanner geometry, analytic
ellipse phantoms, their exact line integrals and Poisson-noised, log-transformed
sinograms.  It holds none of the method's arithmetic (no system matrix, no
projector, no TV term); both the FP64 oracle and the HIP path consume what it
returns, so it is the only code the two share.

Stand-ins.  The paper reconstructs an NCAT thorax phantom, a physical chest
phantom and a Catphan (Sec. 3); none of them is available, so seeded additive
ellipse phantoms of the same size and contrast range take their place.

Geometry conventions (Sec. 2.1 Eq. 1, Sec. 3 scanner description, App. III Eq. A6):

* image ``[ny][nx]``, x fastest; pixel (i, j) is centred at
  ``((i + 1/2 - nx/2) * d, (j + 1/2 - ny/2) * d)`` with ``d = pixel_mm``;
* view ``v`` at angle ``theta_v`` (default ``2*pi*v/V``, equally spaced over a
  full rotation); source at ``-SAD * (cos theta_v, sin theta_v)``;
* equiangular arc detector centred on the source: bin ``b`` looks along
  ``theta_v + beta_b`` with ``beta_b = (b - (B-1)/2 + bin_offset) * dbeta``;
* the sinogram is ``[n_views][n_bins]``, bin fastest.

Randomness: numpy ``PCG64``; phantom seed ``s``, noise seed ``s + 1000``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, asdict
from typing import Optional

import numpy as np

__all__ = [
    "Geometry", "Ellipse", "fan_dbeta", "geometry_small", "geometry_paper",
    "phantom_small", "phantom_paper", "raster", "line_integrals", "noisy_sinogram",
    "make_case", "random_image", "random_sinogram",
]


@dataclass
class Geometry:
    """Fan-beam scanner geometry (Sec. 3; App. III Eq. A6)."""

    nx: int
    ny: int
    pixel_mm: float
    n_views: int
    n_bins: int
    dbeta_rad: float
    sad_mm: float
    sdd_mm: float
    bin_offset: float = 0.0
    view_angles_rad: Optional[np.ndarray] = None

    def angles(self) -> np.ndarray:
        if self.view_angles_rad is not None:
            return np.asarray(self.view_angles_rad, dtype=np.float64)
        return 2.0 * np.pi * np.arange(self.n_views, dtype=np.float64) / self.n_views

    def as_dict(self) -> dict:
        d = asdict(self)
        if self.view_angles_rad is not None:
            d["view_angles_rad"] = np.asarray(self.view_angles_rad, dtype=np.float64)
        return d


@dataclass
class Ellipse:
    """Additive ellipse: value ``mu`` (mm^-1) inside, centre/semi-axes in mm."""

    cx: float
    cy: float
    a: float
    b: float
    angle: float
    mu: float


def fan_dbeta(nx: int, ny: int, pixel_mm: float, sad_mm: float, n_bins: int) -> float:
    """Detector pitch for which the fan just covers the image square.

    The fan half-angle is ``asin(R / SAD)`` with ``R`` the half-diagonal of the
    image, split evenly over ``n_bins`` bins.
    """
    r = 0.5 * pixel_mm * math.hypot(nx, ny)
    return 2.0 * math.asin(r / sad_mm) / n_bins


def geometry_small() -> Geometry:
    """128^2, 30 views, 256 bins, SAD 500 mm, SDD 1000 mm (the small parity case)."""
    return Geometry(128, 128, 1.0, 30, 256, fan_dbeta(128, 128, 1.0, 500.0, 256), 500.0, 1000.0)


def geometry_paper() -> Geometry:
    """512^2, 40 views, 736 bins, SAD 1000 mm, SDD 1500 mm (the paper-scale case)."""
    return Geometry(512, 512, 1.0, 40, 736, fan_dbeta(512, 512, 1.0, 1000.0, 736), 1000.0, 1500.0)


# ----------------------------------------------------------------------------- phantoms

def _inside(e: Ellipse, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    c, s = math.cos(e.angle), math.sin(e.angle)
    dx, dy = x - e.cx, y - e.cy
    u = (c * dx + s * dy) / e.a
    w = (-s * dx + c * dy) / e.b
    return u * u + w * w <= 1.0


def _circle_inside(body: Ellipse, cx: float, cy: float, r: float, shrink: float = 0.95) -> bool:
    t = np.linspace(0.0, 2.0 * np.pi, 256, endpoint=False)
    px, py = cx + r * np.cos(t), cy + r * np.sin(t)
    scaled = Ellipse(body.cx, body.cy, body.a * shrink, body.b * shrink, body.angle, 0.0)
    return bool(np.all(_inside(scaled, px, py)))


def phantom_small(seed: int, n_inserts: int = 9) -> list[Ellipse]:
    """Random ellipse phantom for a 128 mm field: a body plus ``n_inserts`` ellipses.

    Values stay in [0, 0.03] mm^-1: the body takes mu0 ~ U(0.010, 0.020) and each
    insert adds U(-mu0, 0.03 - mu0); insert bounding circles do not overlap and lie
    inside the body.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    half = 64.0
    body = Ellipse(float(rng.uniform(-5, 5)), float(rng.uniform(-5, 5)),
                   float(rng.uniform(0.70, 0.85)) * half, float(rng.uniform(0.55, 0.80)) * half,
                   float(rng.uniform(0, np.pi)), float(rng.uniform(0.010, 0.020)))
    out = [body]
    circles: list[tuple[float, float, float]] = []
    tries = 0
    while len(out) < 1 + n_inserts:
        tries += 1
        if tries > 100000:
            raise RuntimeError("phantom_small: rejection sampling did not converge")
        a = float(rng.uniform(3, 15))
        b = float(rng.uniform(3, 15))
        ang = float(rng.uniform(0, np.pi))
        r = max(a, b)
        cx = float(rng.uniform(body.cx - body.a, body.cx + body.a))
        cy = float(rng.uniform(body.cy - body.a, body.cy + body.a))
        if not _circle_inside(body, cx, cy, r):
            continue
        if any(math.hypot(cx - qx, cy - qy) < r + qr for qx, qy, qr in circles):
            continue
        mu = float(rng.uniform(-body.mu, 0.03 - body.mu))
        circles.append((cx, cy, r))
        out.append(Ellipse(cx, cy, a, b, ang, mu))
    return out


def phantom_paper(seed: int, n_low: int = 6) -> list[Ellipse]:
    """Thorax-like phantom for a 512 mm field with low-contrast inserts.

    Body ellipse 153.6 x 115.2 mm at 0.020 mm^-1 (water), two lungs at -0.015,
    one bone disc (r 10-15 mm) at +0.015 and ``n_low`` low-contrast discs
    (r 5-15 mm) with |contrast| U(0.5 %, 2 %) of 0.020; bounding circles of all
    inserts are disjoint.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    body = Ellipse(0.0, 0.0, 153.6, 115.2, 0.0, 0.020)
    out = [body]
    circles: list[tuple[float, float, float]] = []
    for side in (-1.0, 1.0):
        a = float(rng.uniform(38, 48))
        b = float(rng.uniform(60, 72))
        cx = side * float(rng.uniform(62, 72))
        cy = float(rng.uniform(-8, 8))
        out.append(Ellipse(cx, cy, a, b, float(rng.uniform(-0.2, 0.2)), -0.015))
        circles.append((cx, cy, max(a, b)))

    def place(r: float) -> tuple[float, float]:
        for _ in range(100000):
            cx = float(rng.uniform(-body.a, body.a))
            cy = float(rng.uniform(-body.b, body.b))
            if not _circle_inside(body, cx, cy, r, shrink=0.92):
                continue
            if any(math.hypot(cx - qx, cy - qy) < r + qr + 2.0 for qx, qy, qr in circles):
                continue
            circles.append((cx, cy, r))
            return cx, cy
        raise RuntimeError("phantom_paper: rejection sampling did not converge")

    r = float(rng.uniform(10, 15))
    cx, cy = place(r)
    out.append(Ellipse(cx, cy, r, r, 0.0, 0.015))
    for _ in range(n_low):
        r = float(rng.uniform(5, 15))
        cx, cy = place(r)
        sign = 1.0 if rng.uniform() < 0.5 else -1.0
        out.append(Ellipse(cx, cy, r, r, 0.0, sign * float(rng.uniform(0.005, 0.02)) * 0.020))
    return out


def raster(ellipses: list[Ellipse], nx: int, ny: int, pixel_mm: float, supersample: int = 4) -> np.ndarray:
    """Area-averaged raster of an additive ellipse phantom, ``[ny][nx]`` float64."""
    k = supersample
    off = (np.arange(k) + 0.5) / k
    xs = ((np.arange(nx)[:, None] + off[None, :]).ravel() - 0.5 * nx) * pixel_mm
    ys = ((np.arange(ny)[:, None] + off[None, :]).ravel() - 0.5 * ny) * pixel_mm
    X, Y = np.meshgrid(xs, ys)
    img = np.zeros_like(X)
    for e in ellipses:
        img += e.mu * _inside(e, X, Y)
    return img.reshape(ny, k, nx, k).mean(axis=(1, 3))


def line_integrals(ellipses: list[Ellipse], g: Geometry) -> np.ndarray:
    """Exact line integrals of the phantom along every ray, ``[V][B]`` float64.

    Each ray is the full line through the source with direction
    ``theta_v + beta_b``; its chord through an ellipse is the distance between
    the two roots of the ellipse's quadratic along the line.
    """
    th = g.angles()[:, None]
    beta = (np.arange(g.n_bins)[None, :] - 0.5 * (g.n_bins - 1) + g.bin_offset) * g.dbeta_rad
    sx = -g.sad_mm * np.cos(th)
    sy = -g.sad_mm * np.sin(th)
    dx = np.cos(th + beta)
    dy = np.sin(th + beta)
    sx, sy = np.broadcast_to(sx, dx.shape), np.broadcast_to(sy, dx.shape)
    out = np.zeros(dx.shape)
    for e in ellipses:
        c, s = math.cos(e.angle), math.sin(e.angle)
        px, py = sx - e.cx, sy - e.cy
        pu = (c * px + s * py) / e.a
        pw = (-s * px + c * py) / e.b
        du = (c * dx + s * dy) / e.a
        dw = (-s * dx + c * dy) / e.b
        A = du * du + dw * dw
        Bq = 2.0 * (pu * du + pw * dw)
        C = pu * pu + pw * pw - 1.0
        disc = Bq * Bq - 4.0 * A * C
        out += e.mu * np.sqrt(np.maximum(disc, 0.0)) / A
    return out


def noisy_sinogram(p: np.ndarray, i0: float, seed: int) -> np.ndarray:
    """Poisson counts at ``i0 * exp(-p)``, log-transformed (Sec. 2.1): ``-ln(max(n,1)/i0)``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    counts = rng.poisson(i0 * np.exp(-p)).astype(np.float64)
    return -np.log(np.maximum(counts, 1.0) / i0)


def random_image(nx: int, ny: int, seed: int, lo: float = 0.0, hi: float = 0.03) -> np.ndarray:
    """Uniform random image ``[ny][nx]`` float32 (parity input)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=(ny, nx)).astype(np.float32)


def random_sinogram(n_views: int, n_bins: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Uniform random sinogram ``[V][B]`` float32 (parity input)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, size=(n_views, n_bins)).astype(np.float32)


@dataclass
class Case:
    name: str
    geom: Geometry
    ellipses: list
    phantom: np.ndarray          # [ny][nx] float64, 4x4 supersampled raster
    p: np.ndarray                # [V][B] float64, exact line integrals
    y: np.ndarray                # [V][B] float64, noisy log data
    i0: float
    seed: int
    meta: dict = field(default_factory=dict)


def make_case(name: str, seed: int = 0) -> Case:
    """The two workload shapes: ``"small"`` (128^2/30 views, I0 1e4) and ``"paper"`` (512^2/40 views, I0 5e4)."""
    if name == "small":
        g, ell, i0 = geometry_small(), phantom_small(seed), 1e4
    elif name == "paper":
        g, ell, i0 = geometry_paper(), phantom_paper(seed), 5e4
    else:
        raise ValueError(f"unknown case {name!r}")
    p = line_integrals(ell, g)
    y = noisy_sinogram(p, i0, seed + 1000)
    img = raster(ell, g.nx, g.ny, g.pixel_mm)
    return Case(name, g, ell, img, p, y, i0, seed)


def scaled(ellipses: list[Ellipse], k: float) -> list[Ellipse]:
    """The same phantom with every length multiplied by ``k`` (values kept)."""
    return [Ellipse(e.cx * k, e.cy * k, e.a * k, e.b * k, e.angle, e.mu) for e in ellipses]


def batch_cases(n: int = 64, seed: int = 0, sizes=(256, 384, 512), views=(20, 60), bins=(368, 736),
                i0=(1e4, 1e5), with_phantom: bool = True) -> list[Case]:
    """Slices of uneven size for the batched workload: image side uniform in
    ``sizes`` (1 mm pixels), views uniform in ``views`` (inclusive), bins
    uniform in ``bins`` (inclusive), I0 log-uniform in ``i0``; SAD 1000 mm, SDD
    1500 mm, the fan just covering the image.  Slice ``i`` uses the thorax
    phantom of seed ``seed + i`` (``+ 100000`` until its inserts fit) scaled
    to its field (side / 512), and noise
    seed ``seed + i + 1000``.  The shape draws use PCG64(seed + 50000).
    ``with_phantom=False`` skips the (slow) supersampled raster; the case's
    phantom is then None."""
    rng = np.random.Generator(np.random.PCG64(seed + 50000))
    out = []
    for i in range(n):
        side = int(rng.choice(sizes))
        v = int(rng.integers(views[0], views[1] + 1))
        b = int(rng.integers(bins[0], bins[1] + 1))
        i0_ = float(np.exp(rng.uniform(np.log(i0[0]), np.log(i0[1]))))
        g = Geometry(side, side, 1.0, v, b, fan_dbeta(side, side, 1.0, 1000.0, b), 1000.0, 1500.0)
        ps = seed + i
        while True:  # a few seeds leave no room for the inserts; take the next one
            try:
                ell = scaled(phantom_paper(ps), side / 512.0)
                break
            except RuntimeError:
                ps += 100000
        pr = line_integrals(ell, g)
        y = noisy_sinogram(pr, i0_, seed + i + 1000)
        img = raster(ell, side, side, 1.0) if with_phantom else None
        out.append(Case(f"batch{i}", g, ell, img, pr, y, i0_, seed + i))
    return out
