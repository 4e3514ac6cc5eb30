"""ctypes wrapper of the FP64 CPU oracle (``liboracle.so``).

TEST INFRASTRUCTURE: only the tests, the smoke check and the CPU-baseline leg of
the benchmark may import this module.  It only marshals numpy arrays to the C
library built from ``eptv_oracle.c``; every step of the arithmetic lives there.
It never imports the HIP package and the HIP package never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, asdict
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "eptv_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    """Compile ``liboracle.so`` next to its source (gcc, -O2, no fast-math, OpenMP)."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99", "-Wall",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


class _Geom(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("pixel_mm", C.c_double),
                ("n_views", C.c_int), ("view_angles_rad", C.POINTER(C.c_double)),
                ("n_bins", C.c_int), ("dbeta_rad", C.c_double), ("bin_offset", C.c_double),
                ("sad_mm", C.c_double), ("sdd_mm", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("cgls_iters", C.c_int), ("tv_iters", C.c_int),
                ("zero_init", C.c_int), ("mu", C.c_double), ("lambda_", C.c_double),
                ("edge_quantile", C.c_double), ("sigma_fixed", C.c_double),
                ("sigma_floor", C.c_double), ("tv_eps", C.c_double), ("armijo_c", C.c_double),
                ("armijo_shrink", C.c_double), ("armijo_t0", C.c_double),
                ("armijo_max_backtracks", C.c_int), ("p2_start", C.c_int),
                ("positivity", C.c_int), ("track_energy", C.c_int), ("interp_bp", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("sigma", C.POINTER(C.c_double)), ("armijo_k", C.POINTER(C.c_int)),
                ("armijo_margin", C.POINTER(C.c_double)), ("energy", C.POINTER(C.c_double)),
                ("cgls_steps", C.POINTER(C.c_int)), ("cgls_resid", C.POINTER(C.c_double)),
                ("rmse", C.POINTER(C.c_double)), ("armijo_q0", C.POINTER(C.c_double)),
                ("armijo_q1", C.POINTER(C.c_double)), ("cgls_gamma", C.POINTER(C.c_double)),
                ("cgls_delta", C.POINTER(C.c_double))]


@dataclass
class Params:
    """Solver parameters; the defaults are the readings listed in the design notes."""

    outer_iters: int = 50
    cgls_iters: int = 3
    tv_iters: int = 5
    zero_init: int = 1
    mu: float = 1.0
    lam: float = 1000.0
    edge_quantile: float = 0.90
    sigma_fixed: float = -1.0
    sigma_floor: float = 1e-12
    tv_eps: float = 1e-4
    armijo_c: float = 1e-4
    armijo_shrink: float = 0.5
    armijo_t0: float = 0.0
    armijo_max_backtracks: int = 20
    p2_start: int = 0
    positivity: int = 1
    track_energy: int = 0
    interp_bp: int = 0

    def _c(self) -> _Params:
        d = asdict(self)
        d["lambda_"] = d.pop("lam")
        return _Params(**d)


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        dp, ip = C.POINTER(C.c_double), C.POINTER(C.c_int)
        L.orc_matrix_build.argtypes = [C.POINTER(_Geom), C.POINTER(C.c_void_p)]
        L.orc_matrix_free.argtypes = [C.c_void_p]
        L.orc_matrix_nnz.argtypes = [C.c_void_p]
        L.orc_matrix_nnz.restype = C.c_longlong
        L.orc_matrix_csr.argtypes = [C.c_void_p, C.POINTER(C.c_longlong), ip, dp]
        L.orc_trace_ray.argtypes = [C.POINTER(_Geom), C.c_int, C.c_int, C.c_int, ip, dp]
        L.orc_project.argtypes = [C.c_void_p, dp, dp]
        L.orc_backproject.argtypes = [C.c_void_p, dp, dp]
        L.orc_backproject_interp.argtypes = [C.POINTER(_Geom), dp, dp]
        L.orc_tv_edges.argtypes = [C.c_int, C.c_int, dp, C.c_double, dp, dp]
        L.orc_tv_energy.argtypes = [C.c_int, C.c_int, dp, C.c_double, C.c_double]
        L.orc_tv_energy.restype = C.c_double
        L.orc_tv_gradient.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, C.c_double, C.c_double,
                                      dp, dp, dp]
        L.orc_tv_gradient_vjp.argtypes = [C.c_int, C.c_int, dp, C.c_double, C.c_double, C.c_double, dp, dp]
        L.orc_surrogate.argtypes = [C.c_int, C.c_int, dp, dp, C.c_double, dp, dp, C.c_double]
        L.orc_surrogate.restype = C.c_double
        L.orc_select_sigma.argtypes = [C.c_int, C.c_int, dp, C.c_double, C.c_double, C.c_double]
        L.orc_select_sigma.restype = C.c_double
        L.orc_cgls.argtypes = [C.c_void_p, dp, dp, C.c_int, dp]
        L.orc_cgls_with.argtypes = [C.c_void_p, C.c_int, dp, dp, C.c_int, dp]
        L.orc_tv_step.argtypes = [C.c_int, C.c_int, C.POINTER(_Params), dp, dp, C.c_double, C.c_int,
                                  ip, dp, dp]
        L.orc_reconstruct.argtypes = [C.c_void_p, C.POINTER(_Params), dp, dp, dp, C.POINTER(_Stats)]
        L.orc_reconstruct_weighted.argtypes = [C.c_void_p, C.POINTER(_Params), dp, dp, dp, C.POINTER(_Stats), dp, dp,
                                               C.c_int]
        L.orc_reconstruct_replay.argtypes = [C.c_void_p, C.POINTER(_Params), dp, dp, dp, C.POINTER(_Stats),
                                             C.POINTER(C.c_int)]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _d(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _geom(g) -> tuple[_Geom, Optional[np.ndarray]]:
    ang = getattr(g, "view_angles_rad", None)
    keep = None
    ptr = None
    if ang is not None:
        keep = _f64(ang)
        ptr = _d(keep)
    cg = _Geom(int(g.nx), int(g.ny), float(g.pixel_mm), int(g.n_views), ptr, int(g.n_bins),
               float(g.dbeta_rad), float(getattr(g, "bin_offset", 0.0)), float(g.sad_mm),
               float(g.sdd_mm))
    return cg, keep


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops from now on (timing only: the
    results do not depend on it)."""
    lib().orc_set_num_threads(int(n))


def backproject_interp(g, r) -> np.ndarray:
    """Eq. 11 (App. III): pixel-driven backprojection with linear interpolation in beta."""
    r = _f64(r).reshape(-1)
    assert r.size == int(g.n_views) * int(g.n_bins)
    cg, keep = _geom(g)
    z = np.zeros(int(g.nx) * int(g.ny))
    lib().orc_backproject_interp(C.byref(cg), _d(r), _d(z))
    del keep
    return z.reshape(int(g.ny), int(g.nx))


class Matrix:
    """The system matrix P of a geometry (Sec. 2.1 Eq. 1), held by the C library."""

    def __init__(self, g):
        self.g = g
        self.nx, self.ny = int(g.nx), int(g.ny)
        self.n_views, self.n_bins = int(g.n_views), int(g.n_bins)
        cg, self._keep = _geom(g)
        h = C.c_void_p()
        rc = lib().orc_matrix_build(C.byref(cg), C.byref(h))
        if rc != 0:
            raise ValueError(f"orc_matrix_build failed ({rc})")
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.orc_matrix_free(h)
            self._h = None

    @property
    def nnz(self) -> int:
        return int(lib().orc_matrix_nnz(self._h))

    def csr(self):
        n = self.nnz
        rp = np.zeros(self.n_views * self.n_bins + 1, np.int64)
        col = np.zeros(n, np.int32)
        val = np.zeros(n, np.float64)
        lib().orc_matrix_csr(self._h, rp.ctypes.data_as(C.POINTER(C.c_longlong)), _i(col), _d(val))
        return rp, col, val

    def project(self, x) -> np.ndarray:
        x = _f64(x).reshape(-1)
        assert x.size == self.nx * self.ny
        q = np.zeros(self.n_views * self.n_bins)
        lib().orc_project(self._h, _d(x), _d(q))
        return q.reshape(self.n_views, self.n_bins)

    def backproject(self, r) -> np.ndarray:
        r = _f64(r).reshape(-1)
        assert r.size == self.n_views * self.n_bins
        z = np.zeros(self.nx * self.ny)
        lib().orc_backproject(self._h, _d(r), _d(z))
        return z.reshape(self.ny, self.nx)

    def backproject_interp(self, r) -> np.ndarray:
        """The Eq. 11 backprojector of the same geometry."""
        return backproject_interp(self.g, r)

    def cgls(self, y, u0, iters: int, interp_bp: int = 0):
        u = _f64(u0).reshape(-1).copy()
        res = np.zeros(1)
        steps = lib().orc_cgls_with(self._h, int(interp_bp), _d(_f64(y).reshape(-1)), _d(u), int(iters),
                                    _d(res))
        return u.reshape(self.ny, self.nx), int(steps), float(res[0])

    def reconstruct(self, y, params: Params, f0=None, f_ref=None, weights=None,
                    frozen_iters: int = 0, armijo_replay=None) -> tuple[np.ndarray, dict]:
        """weights: optional (wx [ny][nx+1], wy [ny+1][nx]) used in place of
        Eq. 5's weights during the first frozen_iters iterations.
        armijo_replay: optional [K][T] backtrack indices (-1: no step) taken
        instead of searching; armijo_margin then holds the signed
        certification of each (>= 0: the oracle's own search agrees)."""
        K, T, M = params.outer_iters, params.tv_iters, params.cgls_iters
        f = np.zeros(self.nx * self.ny) if f0 is None else _f64(f0).reshape(-1).copy()
        st = {"sigma": np.zeros(K), "armijo_k": np.zeros(max(K * T, 1), np.int32),
              "armijo_margin": np.zeros(max(K * T, 1)), "energy": np.zeros(K),
              "cgls_steps": np.zeros(K, np.int32), "cgls_resid": np.zeros(K), "rmse": np.zeros(K),
              "armijo_q0": np.zeros(max(K * T, 1)), "armijo_q1": np.zeros(max(K * T, 1)),
              "cgls_gamma": np.zeros(max(K * M, 1)), "cgls_delta": np.zeros(max(K * M, 1))}
        cs = _Stats(_d(st["sigma"]), _i(st["armijo_k"]), _d(st["armijo_margin"]), _d(st["energy"]),
                    _i(st["cgls_steps"]), _d(st["cgls_resid"]), _d(st["rmse"]), _d(st["armijo_q0"]),
                    _d(st["armijo_q1"]), _d(st["cgls_gamma"]), _d(st["cgls_delta"]))
        ref = _f64(f_ref).reshape(-1) if f_ref is not None else None
        cp = params._c()
        if armijo_replay is not None:
            assert weights is None
            rp = np.ascontiguousarray(np.asarray(armijo_replay, dtype=np.int32).reshape(-1))
            assert rp.size == K * T
            rc = lib().orc_reconstruct_replay(self._h, C.byref(cp), _d(_f64(y).reshape(-1)), _d(f),
                                              _d(ref) if ref is not None else None, C.byref(cs), _i(rp))
        elif weights is not None:
            wx, wy = _f64(weights[0]), _f64(weights[1])
            assert wx.shape == (self.ny, self.nx + 1) and wy.shape == (self.ny + 1, self.nx)
            rc = lib().orc_reconstruct_weighted(self._h, C.byref(cp), _d(_f64(y).reshape(-1)), _d(f),
                                                _d(ref) if ref is not None else None, C.byref(cs), _d(wx), _d(wy),
                                                int(frozen_iters))
        else:
            rc = lib().orc_reconstruct(self._h, C.byref(cp), _d(_f64(y).reshape(-1)), _d(f),
                                       _d(ref) if ref is not None else None, C.byref(cs))
        if rc != 0:
            raise ValueError(f"orc_reconstruct failed ({rc})")
        for key in ("armijo_k", "armijo_margin", "armijo_q0", "armijo_q1"):
            st[key] = st[key][:K * T].reshape(K, T)
        for key in ("cgls_gamma", "cgls_delta"):
            st[key] = st[key][:K * M].reshape(K, M)
        if ref is None:
            st.pop("rmse")
        return f.reshape(self.ny, self.nx), st


def trace_ray(g, v: int, b: int):
    cg, keep = _geom(g)
    cap = int(g.nx) + int(g.ny) + 4
    pix = np.zeros(cap, np.int32)
    ln = np.zeros(cap)
    n = lib().orc_trace_ray(C.byref(cg), int(v), int(b), cap, _i(pix), _d(ln))
    return pix[:n].copy(), ln[:n].copy()


def tv_edges(f, eps: float):
    f = _f64(f)
    ny, nx = f.shape
    tvx = np.zeros((ny, nx + 1))
    tvy = np.zeros((ny + 1, nx))
    lib().orc_tv_edges(nx, ny, _d(f), float(eps), _d(tvx), _d(tvy))
    return tvx, tvy


def tv_energy(f, sigma: float, eps: float) -> float:
    f = _f64(f)
    ny, nx = f.shape
    return float(lib().orc_tv_energy(nx, ny, _d(f), float(sigma), float(eps)))


def tv_gradient(f, v, lam: float, sigma: float, eps: float):
    """Returns (g, wx, wy): the P2 direction of Eq. 9 and the half-edge weights at f."""
    f, v = _f64(f), _f64(v)
    ny, nx = f.shape
    g = np.zeros((ny, nx))
    wx = np.zeros((ny, nx + 1))
    wy = np.zeros((ny + 1, nx))
    lib().orc_tv_gradient(nx, ny, _d(f), _d(v), float(lam), float(sigma), float(eps), _d(g), _d(wx), _d(wy))
    return g, wx, wy


def tv_gradient_vjp(f, u, lam: float, sigma: float, eps: float) -> np.ndarray:
    """(dg/df)^T u for the P2 direction g of Eq. 9 (sigma fixed)."""
    f, u = _f64(f), _f64(u)
    ny, nx = f.shape
    out = np.zeros((ny, nx))
    lib().orc_tv_gradient_vjp(nx, ny, _d(f), float(lam), float(sigma), float(eps), _d(u), _d(out))
    return out


def surrogate(h, v, lam: float, wx, wy, eps: float) -> float:
    h, v = _f64(h), _f64(v)
    ny, nx = h.shape
    return float(lib().orc_surrogate(nx, ny, _d(h), _d(v), float(lam), _d(_f64(wx)), _d(_f64(wy)), float(eps)))


def select_sigma(f, eps: float, q: float, floor: float = 1e-12) -> float:
    f = _f64(f)
    ny, nx = f.shape
    return float(lib().orc_select_sigma(nx, ny, _d(f), float(eps), float(q), float(floor)))


def tv_step(f, v, params: Params, n_steps: int, sigma: float = -1.0):
    """P2 descent steps from f towards v. Returns (f_new, k_per_step, margin_per_step, sigma)."""
    f = _f64(f).copy()
    v = _f64(v)
    ny, nx = f.shape
    ks = np.zeros(max(n_steps, 1), np.int32)
    ms = np.zeros(max(n_steps, 1))
    so = np.zeros(1)
    cp = params._c()
    lib().orc_tv_step(nx, ny, C.byref(cp), _d(f), _d(v), float(sigma), int(n_steps), _i(ks), _d(ms), _d(so))
    return f, ks[:n_steps].copy(), ms[:n_steps].copy(), float(so[0])
