"""Python binding of ``libeptv.so`` (the C ABI declared in ``include/eptv.h``).

Argument marshalling only: tensors are checked (float32, contiguous, on the
plan's GPU, right shape) and their device pointers passed to the library; every
step of the computation runs in the library's HIP kernels.  PyTorch provides
device memory and streams.  There is no fallback: if the library is not built
or no GPU is present the calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass, asdict
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libeptv.so")

EPTV_OK, EPTV_ERR_ARG, EPTV_ERR_GEOMETRY, EPTV_ERR_WORKSPACE, EPTV_ERR_HIP, EPTV_ERR_NONFINITE = range(6)

SYMBOLS = ["eptv_plan_create", "eptv_plan_destroy", "eptv_plan_nnz", "eptv_workspace_bytes", "eptv_project",
           "eptv_project_dual", "eptv_backproject", "eptv_tv_gradient", "eptv_select_sigma", "eptv_tv_step", "eptv_reconstruct",
           "eptv_status_string", "eptv_last_error", "eptv_geometry_matrix", "eptv_plan_store_matrix",
           "eptv_plan_stored_layout",
           "eptv_project_stored", "eptv_project_stored_dual", "eptv_backproject_stored", "eptv_backproject_interp",
           "eptv_tv_gradient_vjp", "eptv_batch_create", "eptv_batch_destroy", "eptv_batch_size", "eptv_batch_plan",
           "eptv_batch_workspace_bytes", "eptv_batch_set_launch", "eptv_batch_get_launch", "eptv_batch_tune",
           "eptv_batch_reconstruct", "eptv_unet_create", "eptv_unet_destroy", "eptv_unet_param_count",
           "eptv_unet_set_params", "eptv_unet_get_params", "eptv_unet_get_grads", "eptv_unet_forward",
           "eptv_unet_backward", "eptv_unet_adam", "eptv_unet_mse", "eptv_reconstruct_weighted",
           "eptv_maps_from_eptv", "eptv_maps_to_eptv", "eptv_reconstruct_replay",
           "eptv_reconstruct_noalloc", "eptv_noalloc_scratch_bytes", "eptv_stream_read",
           "eptv_batch_operator_workspace_bytes", "eptv_batch_project", "eptv_batch_backproject"]


class EptvError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = f"{where}: {_lib().eptv_status_string(status).decode()}"
        extra = _lib().eptv_last_error().decode()
        if status == EPTV_ERR_HIP and extra:
            msg += f" ({extra})"
        super().__init__(msg)


class _Geometry(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("pixel_mm", C.c_double), ("n_views", C.c_int),
                ("view_angles_rad", C.POINTER(C.c_double)), ("n_bins", C.c_int), ("dbeta_rad", C.c_double),
                ("bin_offset", C.c_double), ("sad_mm", C.c_double), ("sdd_mm", C.c_double)]


class _Params(C.Structure):
    _fields_ = [("outer_iters", C.c_int), ("cgls_iters", C.c_int), ("tv_iters", C.c_int), ("zero_init", C.c_int),
                ("mu", C.c_double), ("lambda_", C.c_double), ("edge_quantile", C.c_double),
                ("sigma_fixed", C.c_double), ("sigma_floor", C.c_double), ("tv_eps", C.c_double),
                ("armijo_c", C.c_double), ("armijo_shrink", C.c_double), ("armijo_t0", C.c_double),
                ("armijo_max_backtracks", C.c_int), ("p2_start", C.c_int), ("positivity", C.c_int),
                ("stored_matrix", C.c_int), ("interp_bp", C.c_int), ("check_every", C.c_int),
                ("stop_rmse", C.c_double), ("check_finite", C.c_int)]


class _Stats(C.Structure):
    _fields_ = [("sigma", C.POINTER(C.c_float)), ("armijo_k", C.POINTER(C.c_int32)),
                ("cgls_steps", C.POINTER(C.c_int32)), ("cgls_resid", C.POINTER(C.c_double)),
                ("rmse", C.POINTER(C.c_double)), ("iters_run", C.POINTER(C.c_int32)),
                ("armijo_q0", C.POINTER(C.c_double)), ("armijo_q1", C.POINTER(C.c_double)),
                ("cgls_gamma", C.POINTER(C.c_double)), ("cgls_delta", C.POINTER(C.c_double))]


def _records(K: int, T: int, M: int) -> dict:
    """Host arrays for every per-iteration record of eptv_stats."""
    import numpy as np
    return {"sigma": np.zeros(max(K, 1), np.float32), "armijo_k": np.zeros(max(K * T, 1), np.int32),
            "cgls_steps": np.zeros(max(K, 1), np.int32), "cgls_resid": np.zeros(max(K, 1)),
            "rmse": np.zeros(max(K, 1)), "armijo_q0": np.zeros(max(K * T, 1)), "armijo_q1": np.zeros(max(K * T, 1)),
            "cgls_gamma": np.zeros(max(K * M, 1)), "cgls_delta": np.zeros(max(K * M, 1))}


def _stats_of(rec: dict, done=None) -> "_Stats":
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))  # noqa: E731
    return _Stats(rec["sigma"].ctypes.data_as(C.POINTER(C.c_float)),
                  rec["armijo_k"].ctypes.data_as(C.POINTER(C.c_int32)),
                  rec["cgls_steps"].ctypes.data_as(C.POINTER(C.c_int32)), dp(rec["cgls_resid"]), dp(rec["rmse"]),
                  done.ctypes.data_as(C.POINTER(C.c_int32)) if done is not None else None, dp(rec["armijo_q0"]),
                  dp(rec["armijo_q1"]), dp(rec["cgls_gamma"]), dp(rec["cgls_delta"]))


def _shape_records(rec: dict, n: int, T: int, M: int) -> dict:
    """The first n iterations' records, per-step ones as [n][T] / [n][M]."""
    out = {k: v[:n].copy() for k, v in rec.items() if k not in ("armijo_k", "armijo_q0", "armijo_q1",
                                                                  "cgls_gamma", "cgls_delta")}
    for k in ("armijo_k", "armijo_q0", "armijo_q1"):
        out[k] = rec[k][:n * T].reshape(n, T).copy()
    for k in ("cgls_gamma", "cgls_delta"):
        out[k] = rec[k][:n * M].reshape(n, M).copy()
    return out


@dataclass
class Params:
    """Solver parameters (the fields of ``eptv_params``)."""

    outer_iters: int = 100
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
    stored_matrix: int = 0
    interp_bp: int = 0
    check_every: int = 1
    stop_rmse: float = 0.0
    check_finite: int = 0

    def _c(self) -> _Params:
        d = asdict(self)
        d["lambda_"] = d.pop("lam")
        return _Params(**d)


_L = None


def _lib() -> C.CDLL:
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1009_2288_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, sz = C.c_void_p, C.c_size_t
        L.eptv_plan_create.argtypes = [C.POINTER(_Geometry), C.POINTER(vp)]
        L.eptv_plan_destroy.argtypes = [vp]
        L.eptv_plan_nnz.argtypes = [vp, C.POINTER(C.c_longlong)]
        L.eptv_workspace_bytes.argtypes = [vp, C.POINTER(_Params), C.POINTER(sz)]
        L.eptv_project.argtypes = [vp, vp, vp, C.c_float, C.c_float, vp, sz, vp]
        L.eptv_project_dual.argtypes = [vp, vp, vp, vp, C.c_float, C.c_float, vp]
        L.eptv_backproject.argtypes = [vp, vp, vp, C.c_float, C.c_float, vp, sz, vp]
        L.eptv_tv_gradient.argtypes = [vp, vp, vp, C.c_float, C.c_float, C.c_float, vp, vp, vp, vp, sz, vp]
        L.eptv_batch_create.argtypes = [C.POINTER(_Geometry), C.c_int, C.POINTER(vp)]
        L.eptv_batch_destroy.argtypes = [vp]
        L.eptv_batch_size.argtypes = [vp, C.POINTER(C.c_int)]
        L.eptv_batch_plan.argtypes = [vp, C.c_int, C.POINTER(vp)]
        L.eptv_batch_workspace_bytes.argtypes = [vp, C.POINTER(_Params), C.POINTER(sz)]
        L.eptv_batch_set_launch.argtypes = [vp, C.c_int, C.c_int, C.c_int]
        L.eptv_batch_get_launch.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
        L.eptv_batch_tune.argtypes = [vp, C.c_int, vp, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.eptv_batch_reconstruct.argtypes = [vp, C.POINTER(_Params), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp,
                                             sz, C.POINTER(_Stats), vp]
        L.eptv_unet_create.argtypes = [C.c_int] * 7 + [C.POINTER(vp)]
        L.eptv_unet_destroy.argtypes = [vp]
        L.eptv_unet_param_count.argtypes = [vp, C.POINTER(C.c_longlong)]
        L.eptv_unet_set_params.argtypes = [vp, vp, vp]
        L.eptv_unet_get_params.argtypes = [vp, vp, vp]
        L.eptv_unet_get_grads.argtypes = [vp, vp, vp]
        L.eptv_unet_forward.argtypes = [vp, vp, C.c_int, vp, vp]
        L.eptv_unet_backward.argtypes = [vp, vp, vp, vp]
        L.eptv_unet_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int, vp]
        L.eptv_unet_mse.argtypes = [vp, vp, vp, sz, vp, vp, vp]
        L.eptv_maps_from_eptv.argtypes = [C.c_int, C.c_int, C.c_int, vp, vp, vp, vp, C.c_float, vp, vp]
        L.eptv_maps_to_eptv.argtypes = [C.c_int, C.c_int, C.c_int, vp, C.c_float, vp, vp, vp, vp, vp]
        L.eptv_tv_gradient_vjp.argtypes = [vp, vp, vp, C.c_float, C.c_float, C.c_float, vp, vp, sz, vp]
        L.eptv_select_sigma.argtypes = [vp, vp, C.c_double, C.c_float, C.c_float, vp, vp, sz, vp]
        L.eptv_tv_step.argtypes = [vp, C.POINTER(_Params), vp, vp, C.c_float, C.c_int, vp, sz, C.POINTER(_Stats), vp]
        L.eptv_reconstruct.argtypes = [vp, C.POINTER(_Params), vp, vp, vp, vp, sz, C.POINTER(_Stats), vp]
        L.eptv_reconstruct_noalloc.argtypes = [vp, C.POINTER(_Params), vp, vp, vp, C.POINTER(_Stats), vp]
        L.eptv_noalloc_scratch_bytes.argtypes = []
        L.eptv_noalloc_scratch_bytes.restype = sz
        L.eptv_stream_read.argtypes = [vp, sz, vp, vp]
        L.eptv_batch_operator_workspace_bytes.argtypes = [vp, C.POINTER(sz)]
        L.eptv_batch_project.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.c_float, C.c_float, vp, sz, vp]
        L.eptv_batch_backproject.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.c_float, C.c_float, vp, sz, vp]
        L.eptv_reconstruct_replay.argtypes = [vp, C.POINTER(_Params), vp, vp, vp, C.POINTER(C.c_int32), vp, sz,
                                              C.POINTER(_Stats), vp]
        L.eptv_reconstruct_weighted.argtypes = [vp, C.POINTER(_Params), vp, vp, vp, vp, vp, C.c_int, vp, sz,
                                                C.POINTER(_Stats), vp]
        L.eptv_geometry_matrix.argtypes = [C.POINTER(_Geometry), C.POINTER(C.c_longlong), vp, vp, vp]
        L.eptv_plan_store_matrix.argtypes = [vp, C.POINTER(sz)]
        L.eptv_plan_stored_layout.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(sz), C.POINTER(sz)]
        L.eptv_project_stored.argtypes = [vp, vp, vp, C.c_float, C.c_float, vp, sz, vp]
        L.eptv_project_stored_dual.argtypes = [vp, vp, vp, vp, C.c_float, C.c_float, vp]
        L.eptv_backproject_stored.argtypes = [vp, vp, vp, C.c_float, C.c_float, vp]
        L.eptv_backproject_interp.argtypes = [vp, vp, vp, C.c_float, C.c_float, vp]
        L.eptv_status_string.argtypes = [C.c_int]
        L.eptv_status_string.restype = C.c_char_p
        L.eptv_last_error.restype = C.c_char_p
        _L = L
    return _L


def library() -> C.CDLL:
    """The loaded ``libeptv.so`` (raises if it is not built)."""
    return _lib()


def _check(rc: int, where: str) -> None:
    if rc != EPTV_OK:
        raise EptvError(rc, where)


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _geometry(geom):
    """(ctypes struct, keep-alive array) for a geometry object."""
    import numpy as np
    ang = getattr(geom, "view_angles_rad", None)
    keep = None
    ptr = None
    if ang is not None:
        keep = np.ascontiguousarray(np.asarray(ang, dtype=np.float64))
        ptr = keep.ctypes.data_as(C.POINTER(C.c_double))
    g = _Geometry(int(geom.nx), int(geom.ny), float(geom.pixel_mm), int(geom.n_views), ptr, int(geom.n_bins),
                  float(geom.dbeta_rad), float(getattr(geom, "bin_offset", 0.0)), float(geom.sad_mm),
                  float(geom.sdd_mm))
    return g, keep


def geometry_matrix(geom):
    """The float32 system matrix the kernels evaluate, as host CSR arrays
    (rowptr int64, col int32, val float32), computed on the host (no GPU)."""
    import numpy as np
    g, keep = _geometry(geom)
    n = C.c_longlong()
    _check(_lib().eptv_geometry_matrix(C.byref(g), C.byref(n), None, None, None), "eptv_geometry_matrix")
    rp = np.zeros(int(geom.n_views) * int(geom.n_bins) + 1, np.int64)
    col = np.zeros(n.value, np.int32)
    val = np.zeros(n.value, np.float32)
    _check(_lib().eptv_geometry_matrix(C.byref(g), C.byref(n), rp.ctypes.data, col.ctypes.data, val.ctypes.data),
           "eptv_geometry_matrix")
    del keep
    return rp, col, val


class Plan:
    """Geometry tables of one scanner geometry on one GPU (``eptv_plan``)."""

    def __init__(self, geom, device: Optional[torch.device] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("libeptv needs a ROCm GPU; none is visible")
        self.device = torch.device(device if device is not None else "cuda", )
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.nx, self.ny = int(geom.nx), int(geom.ny)
        self.n_views, self.n_bins = int(geom.n_views), int(geom.n_bins)
        g, self._ang = _geometry(geom)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib().eptv_plan_create(C.byref(g), C.byref(h)), "eptv_plan_create")
        self._h = h
        self._ws = None

    @classmethod
    def _borrow(cls, handle, geom, device, owner) -> "Plan":
        """A Plan object for a plan owned by someone else (a batch slice)."""
        self = cls.__new__(cls)
        self.device = device
        self.nx, self.ny = int(geom.nx), int(geom.ny)
        self.n_views, self.n_bins = int(geom.n_views), int(geom.n_bins)
        self._ang = None
        self._h = handle
        self._ws = None
        self._owner = owner
        return self

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _L is not None and getattr(self, "_owner", None) is None:
            _L.eptv_plan_destroy(h)
        self._h = None

    # ------------------------------------------------------------- helpers
    @property
    def nnz(self) -> int:
        n = C.c_longlong()
        _check(_lib().eptv_plan_nnz(self._h, C.byref(n)), "eptv_plan_nnz")
        return int(n.value)

    def workspace_bytes(self, params: Optional[Params] = None) -> int:
        n = C.c_size_t()
        cp = params._c() if params is not None else None
        _check(_lib().eptv_workspace_bytes(self._h, C.byref(cp) if cp is not None else None, C.byref(n)),
               "eptv_workspace_bytes")
        return int(n.value)

    def workspace(self, params: Optional[Params] = None) -> torch.Tensor:
        need = self.workspace_bytes(params)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws

    def _img(self, t: torch.Tensor, name: str) -> torch.Tensor:
        return self._t(t, (self.ny, self.nx), name)

    def _sino(self, t: torch.Tensor, name: str) -> torch.Tensor:
        return self._t(t, (self.n_views, self.n_bins), name)

    def _t(self, t: torch.Tensor, shape, name: str) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.device != self.device:
            raise TypeError(f"{name} must be a float32 tensor on {self.device}")
        if tuple(t.shape) != tuple(shape) or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def new_image(self) -> torch.Tensor:
        return torch.empty((self.ny, self.nx), dtype=torch.float32, device=self.device)

    def new_sinogram(self) -> torch.Tensor:
        return torch.empty((self.n_views, self.n_bins), dtype=torch.float32, device=self.device)

    # ------------------------------------------------------------- the calls
    def project(self, x: torch.Tensor, out: Optional[torch.Tensor] = None, alpha: float = 1.0, beta: float = 0.0,
                stream=None) -> torch.Tensor:
        """out = alpha P x + beta out."""
        x = self._img(x, "x")
        out = self._sino(out if out is not None else self.new_sinogram(), "out")
        ws = self.workspace()
        _check(_lib().eptv_project(self._h, x.data_ptr(), out.data_ptr(), alpha, beta, ws.data_ptr(), ws.numel(),
                                   _stream(stream)), "eptv_project")
        return out

    def project_dual(self, x: torch.Tensor, xT: torch.Tensor, out: Optional[torch.Tensor] = None,
                     alpha: float = 1.0, beta: float = 0.0, stream=None) -> torch.Tensor:
        """out = alpha P x + beta out, with xT the same image transposed ([nx][ny])."""
        x = self._img(x, "x")
        xT = self._t(xT, (self.nx, self.ny), "xT")
        out = self._sino(out if out is not None else self.new_sinogram(), "out")
        _check(_lib().eptv_project_dual(self._h, x.data_ptr(), xT.data_ptr(), out.data_ptr(), alpha, beta,
                                        _stream(stream)), "eptv_project_dual")
        return out

    def store_matrix(self) -> int:
        """Keep the float32 system matrix on the device (CSR + CSC); returns its bytes."""
        n = C.c_size_t()
        with torch.cuda.device(self.device):
            _check(_lib().eptv_plan_store_matrix(self._h, C.byref(n)), "eptv_plan_store_matrix")
        return int(n.value)

    def stored_layout(self) -> dict:
        """The stored matrix's CSR encoding (compact: 6 bytes per entry, else 8)
        and each copy's device bytes."""
        cp, rb, cb = C.c_int(), C.c_size_t(), C.c_size_t()
        _check(_lib().eptv_plan_stored_layout(self._h, C.byref(cp), C.byref(rb), C.byref(cb)),
               "eptv_plan_stored_layout")
        return {"csr_compact": bool(cp.value), "csr_bytes": int(rb.value), "csc_bytes": int(cb.value)}

    def project_stored(self, x: torch.Tensor, out: Optional[torch.Tensor] = None, alpha: float = 1.0,
                       beta: float = 0.0, stream=None) -> torch.Tensor:
        """out = alpha P x + beta out from the stored matrix."""
        x = self._img(x, "x")
        out = self._sino(out if out is not None else self.new_sinogram(), "out")
        ws = self.workspace()
        _check(_lib().eptv_project_stored(self._h, x.data_ptr(), out.data_ptr(), alpha, beta, ws.data_ptr(),
                                          ws.numel(), _stream(stream)), "eptv_project_stored")
        return out

    def project_stored_dual(self, x: torch.Tensor, xT: torch.Tensor, out: Optional[torch.Tensor] = None,
                            alpha: float = 1.0, beta: float = 0.0, stream=None) -> torch.Tensor:
        """project_stored with xT the same image transposed ([nx][ny])."""
        x = self._img(x, "x")
        xT = self._t(xT, (self.nx, self.ny), "xT")
        out = self._sino(out if out is not None else self.new_sinogram(), "out")
        _check(_lib().eptv_project_stored_dual(self._h, x.data_ptr(), xT.data_ptr(), out.data_ptr(), alpha, beta,
                                               _stream(stream)), "eptv_project_stored_dual")
        return out

    def backproject_stored(self, r: torch.Tensor, out: Optional[torch.Tensor] = None, alpha: float = 1.0,
                           beta: float = 0.0, stream=None) -> torch.Tensor:
        r = self._sino(r, "r")
        out = self._img(out if out is not None else self.new_image(), "out")
        _check(_lib().eptv_backproject_stored(self._h, r.data_ptr(), out.data_ptr(), alpha, beta, _stream(stream)),
               "eptv_backproject_stored")
        return out

    def backproject_interp(self, r: torch.Tensor, out: Optional[torch.Tensor] = None, alpha: float = 1.0,
                           beta: float = 0.0, stream=None) -> torch.Tensor:
        """out = alpha B r + beta out, B the Eq. 11 interpolating backprojector."""
        r = self._sino(r, "r")
        out = self._img(out if out is not None else self.new_image(), "out")
        _check(_lib().eptv_backproject_interp(self._h, r.data_ptr(), out.data_ptr(), alpha, beta, _stream(stream)),
               "eptv_backproject_interp")
        return out

    def backproject(self, r: torch.Tensor, out: Optional[torch.Tensor] = None, alpha: float = 1.0,
                    beta: float = 0.0, stream=None) -> torch.Tensor:
        """out = alpha P^T r + beta out."""
        r = self._sino(r, "r")
        out = self._img(out if out is not None else self.new_image(), "out")
        ws = self.workspace()
        _check(_lib().eptv_backproject(self._h, r.data_ptr(), out.data_ptr(), alpha, beta, ws.data_ptr(),
                                       ws.numel(), _stream(stream)), "eptv_backproject")
        return out

    def tv_gradient(self, f: torch.Tensor, v: torch.Tensor, lam: float, sigma: float, tv_eps: float,
                    with_weights: bool = True, stream=None):
        """(g, wx, wy): the P2 direction and the half-edge weights at f."""
        f, v = self._img(f, "f"), self._img(v, "v")
        g = self.new_image()
        wx = torch.empty((self.ny, self.nx + 1), dtype=torch.float32, device=self.device) if with_weights else None
        wy = torch.empty((self.ny + 1, self.nx), dtype=torch.float32, device=self.device) if with_weights else None
        ws = self.workspace()
        _check(_lib().eptv_tv_gradient(self._h, f.data_ptr(), v.data_ptr(), lam, sigma, tv_eps, g.data_ptr(),
                                       wx.data_ptr() if wx is not None else None,
                                       wy.data_ptr() if wy is not None else None, ws.data_ptr(), ws.numel(),
                                       _stream(stream)), "eptv_tv_gradient")
        return g, wx, wy

    def tv_gradient_vjp(self, f: torch.Tensor, u: torch.Tensor, lam: float, sigma: float, tv_eps: float,
                        out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """(dg/df)^T u for the P2 direction g at f (sigma fixed)."""
        f, u = self._img(f, "f"), self._img(u, "u")
        out = self._img(out if out is not None else self.new_image(), "out")
        ws = self.workspace()
        _check(_lib().eptv_tv_gradient_vjp(self._h, f.data_ptr(), u.data_ptr(), lam, sigma, tv_eps, out.data_ptr(),
                                           ws.data_ptr(), ws.numel(), _stream(stream)), "eptv_tv_gradient_vjp")
        return out

    def select_sigma(self, f: torch.Tensor, q: float, tv_eps: float, sigma_floor: float = 1e-12,
                     stream=None) -> torch.Tensor:
        """Device scalar (1-element tensor) holding sigma."""
        f = self._img(f, "f")
        out = torch.empty(1, dtype=torch.float32, device=self.device)
        ws = self.workspace()
        _check(_lib().eptv_select_sigma(self._h, f.data_ptr(), q, tv_eps, sigma_floor, out.data_ptr(),
                                        ws.data_ptr(), ws.numel(), _stream(stream)), "eptv_select_sigma")
        return out

    def tv_step(self, f: torch.Tensor, v: torch.Tensor, params: Params, n_steps: int, sigma: float = -1.0,
                stats: bool = True, stream=None):
        """In-place P2 descent steps on f; returns (armijo_k per step, sigma) when stats."""
        import numpy as np
        f, v = self._img(f, "f"), self._img(v, "v")
        ws = self.workspace()
        ks = np.zeros(max(n_steps, 1), np.int32)
        sg = np.zeros(1, np.float32)
        q0 = np.zeros(max(n_steps, 1))
        q1 = np.zeros(max(n_steps, 1))
        dp = C.POINTER(C.c_double)
        st = _Stats(sg.ctypes.data_as(C.POINTER(C.c_float)), ks.ctypes.data_as(C.POINTER(C.c_int32)), None, None,
                    None, None, q0.ctypes.data_as(dp), q1.ctypes.data_as(dp), None, None)
        cp = params._c()
        _check(_lib().eptv_tv_step(self._h, C.byref(cp), f.data_ptr(), v.data_ptr(), sigma, n_steps, ws.data_ptr(),
                                   ws.numel(), C.byref(st) if stats else None, _stream(stream)), "eptv_tv_step")
        self.last_tv_step_energies = (q0[:n_steps].copy(), q1[:n_steps].copy()) if stats else None
        return (ks[:n_steps].copy(), float(sg[0])) if stats else None

    def reconstruct(self, y: torch.Tensor, params: Params, f: Optional[torch.Tensor] = None,
                    f_ref: Optional[torch.Tensor] = None, stats: bool = True, stream=None, weights=None,
                    frozen_iters: int = 0, armijo_replay=None):
        """Run params.outer_iters EPTV iterations (fewer after an early stop,
        params.stop_rmse); returns (f, stats dict or None).
        weights: optional (wx [ny][nx+1], wy [ny+1][nx]) device tensors used in
        place of Eq. 5's weights during the first frozen_iters iterations.
        armijo_replay: optional [K][T] backtrack indices taken instead of the
        line search (eptv_reconstruct_replay)."""
        import numpy as np
        y = self._sino(y, "y")
        if f is None:
            f = torch.zeros((self.ny, self.nx), dtype=torch.float32, device=self.device)
        f = self._img(f, "f")
        if f_ref is not None:
            f_ref = self._img(f_ref, "f_ref")
        ws = self.workspace(params)
        K, T, M = params.outer_iters, params.tv_iters, params.cgls_iters
        rec = None
        stp = None
        done = np.zeros(1, np.int32)
        if stats:
            rec = _records(K, T, M)
            st = _stats_of(rec, done)
            stp = C.byref(st)
        cp = params._c()
        if armijo_replay is not None:
            if weights is not None:
                raise ValueError("armijo_replay and weights cannot be combined")
            rp = np.ascontiguousarray(np.asarray(armijo_replay, dtype=np.int32).reshape(-1))
            if rp.size != K * T:
                raise ValueError(f"armijo_replay must hold outer_iters * tv_iters = {K * T} indices")
            _check(_lib().eptv_reconstruct_replay(self._h, C.byref(cp), y.data_ptr(), f.data_ptr(),
                                                  f_ref.data_ptr() if f_ref is not None else None,
                                                  rp.ctypes.data_as(C.POINTER(C.c_int32)), ws.data_ptr(),
                                                  ws.numel(), stp, _stream(stream)), "eptv_reconstruct_replay")
        elif weights is not None:
            wx = self._t(weights[0], (self.ny, self.nx + 1), "wx")
            wy = self._t(weights[1], (self.ny + 1, self.nx), "wy")
            _check(_lib().eptv_reconstruct_weighted(self._h, C.byref(cp), y.data_ptr(), f.data_ptr(),
                                                    f_ref.data_ptr() if f_ref is not None else None, wx.data_ptr(),
                                                    wy.data_ptr(), int(frozen_iters), ws.data_ptr(), ws.numel(),
                                                    stp, _stream(stream)), "eptv_reconstruct_weighted")
        else:
            _check(_lib().eptv_reconstruct(self._h, C.byref(cp), y.data_ptr(), f.data_ptr(),
                                           f_ref.data_ptr() if f_ref is not None else None, ws.data_ptr(),
                                           ws.numel(), stp, _stream(stream)), "eptv_reconstruct")
        if rec is not None:
            n = int(done[0])  # iterations run (an early stop leaves fewer than K records)
            rec = _shape_records(rec, n, T, M) | {"iters_run": n}
            if f_ref is None:
                rec.pop("rmse")
        return f, rec

    def reconstruct_noalloc(self, y: torch.Tensor, params: Params, f: Optional[torch.Tensor] = None,
                            f_ref: Optional[torch.Tensor] = None, stats: bool = True, stream=None):
        """reconstruct() through eptv_reconstruct_noalloc: no workspace tensor
        is allocated; the library's fixed device array serves instead."""
        import numpy as np
        y = self._sino(y, "y")
        if f is None:
            f = torch.zeros((self.ny, self.nx), dtype=torch.float32, device=self.device)
        f = self._img(f, "f")
        if f_ref is not None:
            f_ref = self._img(f_ref, "f_ref")
        K, T, M = params.outer_iters, params.tv_iters, params.cgls_iters
        rec = None
        stp = None
        done = np.zeros(1, np.int32)
        if stats:
            rec = _records(K, T, M)
            st = _stats_of(rec, done)
            stp = C.byref(st)
        cp = params._c()
        _check(_lib().eptv_reconstruct_noalloc(self._h, C.byref(cp), y.data_ptr(), f.data_ptr(),
                                               f_ref.data_ptr() if f_ref is not None else None, stp,
                                               _stream(stream)), "eptv_reconstruct_noalloc")
        if rec is not None:
            n = int(done[0])
            rec = _shape_records(rec, n, T, M) | {"iters_run": n}
            if f_ref is None:
                rec.pop("rmse")
        return f, rec


def stream_read(buf: torch.Tensor, sink: torch.Tensor, stream=None) -> None:
    """Read every byte of a contiguous device tensor once (eptv_stream_read), a
    measurement aid: the read-only streaming rate of the GPU."""
    if not buf.is_cuda or not buf.is_contiguous() or not sink.is_cuda or sink.dtype != torch.int32:
        raise ValueError("stream_read: contiguous device tensors, sink int32")
    _check(_lib().eptv_stream_read(buf.data_ptr(), buf.numel() * buf.element_size(), sink.data_ptr(),
                                   _stream(stream)), "eptv_stream_read")


def noalloc_scratch_bytes() -> int:
    """Size of the fixed device array eptv_reconstruct_noalloc works in."""
    return int(_lib().eptv_noalloc_scratch_bytes())


class Batch:
    """Slices of different geometries iterated together (``eptv_batch``): every
    phase of an outer iteration is one launch over all slices."""

    def __init__(self, geoms, device: Optional[torch.device] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("libeptv needs a ROCm GPU; none is visible")
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.geoms = list(geoms)
        structs, self._keep = [], []
        for g in self.geoms:
            cg, keep = _geometry(g)
            structs.append(cg)
            self._keep.append(keep)
        arr = (_Geometry * len(structs))(*structs)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            _check(_lib().eptv_batch_create(arr, len(structs), C.byref(h)), "eptv_batch_create")
        self._h = h
        self._ws = None
        self.plans = []
        for i, g in enumerate(self.geoms):
            ph = C.c_void_p()
            _check(_lib().eptv_batch_plan(self._h, i, C.byref(ph)), "eptv_batch_plan")
            self.plans.append(Plan._borrow(ph, g, self.device, self))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _L is not None:
            for p in getattr(self, "plans", []):
                p._h = None
            _L.eptv_batch_destroy(h)
        self._h = None

    def __len__(self) -> int:
        return len(self.geoms)

    def workspace(self, params: Params) -> torch.Tensor:
        n = C.c_size_t()
        cp = params._c()
        _check(_lib().eptv_batch_workspace_bytes(self._h, C.byref(cp), C.byref(n)), "eptv_batch_workspace_bytes")
        if self._ws is None or self._ws.numel() < n.value:
            self._ws = torch.empty(int(n.value), dtype=torch.uint8, device=self.device)
        return self._ws

    def set_launch(self, proj_seg: int, proj_blocks_per_cu: int, tile_blocks_per_cu: int) -> None:
        _check(_lib().eptv_batch_set_launch(self._h, proj_seg, proj_blocks_per_cu, tile_blocks_per_cu),
               "eptv_batch_set_launch")

    def launch(self) -> dict:
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        _check(_lib().eptv_batch_get_launch(self._h, C.byref(a), C.byref(b), C.byref(c)), "eptv_batch_get_launch")
        return {"proj_seg": a.value, "proj_grid": b.value, "tile_grid": c.value}

    def tune(self, reps: int = 10, stream=None) -> dict:
        pm, bm = C.c_float(), C.c_float()
        _check(_lib().eptv_batch_tune(self._h, reps, _stream(stream), C.byref(pm), C.byref(bm)), "eptv_batch_tune")
        return {"project_ms": pm.value, "backproject_ms": bm.value, **self.launch()}

    def _operator(self, forward: bool, xs, outs, alpha: float, beta: float, stream) -> None:
        n = len(self)
        if len(xs) != n or len(outs) != n:
            raise ValueError(f"expected {n} slices")
        if forward:
            xs = [p._img(x, f"x[{i}]") for i, (p, x) in enumerate(zip(self.plans, xs))]
            outs = [p._sino(o, f"q[{i}]") for i, (p, o) in enumerate(zip(self.plans, outs))]
        else:
            xs = [p._sino(x, f"r[{i}]") for i, (p, x) in enumerate(zip(self.plans, xs))]
            outs = [p._img(o, f"z[{i}]") for i, (p, o) in enumerate(zip(self.plans, outs))]
        nb = C.c_size_t()
        _check(_lib().eptv_batch_operator_workspace_bytes(self._h, C.byref(nb)), "eptv_batch_operator_workspace_bytes")
        if self._ws is None or self._ws.numel() < nb.value:
            self._ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        ip = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
        op = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        fn = _lib().eptv_batch_project if forward else _lib().eptv_batch_backproject
        _check(fn(self._h, ip, op, alpha, beta, self._ws.data_ptr(), self._ws.numel(), _stream(stream)),
               "eptv_batch_project" if forward else "eptv_batch_backproject")

    def project(self, xs, outs=None, alpha: float = 1.0, beta: float = 0.0, stream=None):
        """q_i = alpha P_i x_i + beta q_i for every slice in one launch (eptv_batch_project).
        xs: per-slice images, or a [n, ny, nx] tensor when the slices share a shape;
        returns the outputs in the same form."""
        stacked = isinstance(xs, torch.Tensor)
        if outs is None:
            outs = (torch.empty((len(self), self.plans[0].n_views, self.plans[0].n_bins), dtype=torch.float32,
                                device=self.device) if stacked else [p.new_sinogram() for p in self.plans])
        self._operator(True, list(xs), list(outs), alpha, beta, stream)
        return outs

    def backproject(self, rs, outs=None, alpha: float = 1.0, beta: float = 0.0, stream=None):
        """z_i = alpha P_i^T r_i + beta z_i for every slice in one launch (eptv_batch_backproject)."""
        stacked = isinstance(rs, torch.Tensor)
        if outs is None:
            outs = (torch.empty((len(self), self.plans[0].ny, self.plans[0].nx), dtype=torch.float32,
                                device=self.device) if stacked else [p.new_image() for p in self.plans])
        self._operator(False, list(rs), list(outs), alpha, beta, stream)
        return outs

    def reconstruct(self, ys, params: Params, fs=None, f_refs=None, stats: bool = True, stream=None):
        """params.outer_iters iterations on every slice; returns (list of f, list of stats dicts or None)."""
        import numpy as np
        n = len(self)
        ys = [p._sino(y, f"y[{i}]") for i, (p, y) in enumerate(zip(self.plans, ys))]
        if fs is None:
            fs = [torch.zeros((p.ny, p.nx), dtype=torch.float32, device=self.device) for p in self.plans]
        fs = [p._img(f, f"f[{i}]") for i, (p, f) in enumerate(zip(self.plans, fs))]
        if f_refs is not None:
            f_refs = [p._img(r, f"f_ref[{i}]") for i, (p, r) in enumerate(zip(self.plans, f_refs))]
        if len(ys) != n or len(fs) != n or (f_refs is not None and len(f_refs) != n):
            raise ValueError(f"expected {n} slices")
        ws = self.workspace(params)
        K, T, M = params.outer_iters, params.tv_iters, params.cgls_iters
        yp = (C.c_void_p * n)(*[y.data_ptr() for y in ys])
        fp = (C.c_void_p * n)(*[f.data_ptr() for f in fs])
        rp = (C.c_void_p * n)(*[r.data_ptr() for r in f_refs]) if f_refs is not None else None
        recs, sts = None, None
        if stats:
            recs = [_records(K, T, M) for _ in range(n)]
            sts = (_Stats * n)(*[_stats_of(r) for r in recs])
        cp = params._c()
        _check(_lib().eptv_batch_reconstruct(self._h, C.byref(cp), yp, fp, rp, ws.data_ptr(), ws.numel(), sts,
                                             _stream(stream)), "eptv_batch_reconstruct")
        if recs is not None:
            out = []
            for r in recs:
                d = _shape_records(r, K, T, M)
                if f_refs is None:
                    d.pop("rmse")
                out.append(d)
            recs = out
        return fs, recs


class UNet:
    """The edge-weight / warm-start network (``eptv_unet``): bf16 MFMA layers,
    fp32 masters, Adam.  Tensors are float32 NHWC on the GPU."""

    def __init__(self, c_in: int, c_out: int, base: int, levels: int, max_batch: int, height: int, width: int):
        if not torch.cuda.is_available():
            raise RuntimeError("libeptv needs a ROCm GPU; none is visible")
        self.c_in, self.c_out, self.base, self.levels = c_in, c_out, base, levels
        self.max_batch, self.h, self.w = max_batch, height, width
        self.device = torch.device("cuda", torch.cuda.current_device())
        h = C.c_void_p()
        _check(_lib().eptv_unet_create(c_in, c_out, base, levels, max_batch, height, width, C.byref(h)),
               "eptv_unet_create")
        self._h = h
        n = C.c_longlong()
        _check(_lib().eptv_unet_param_count(self._h, C.byref(n)), "eptv_unet_param_count")
        self.n_params = int(n.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _L is not None:
            _L.eptv_unet_destroy(h)
        self._h = None

    def set_params(self, flat, stream=None) -> None:
        import numpy as np
        a = np.ascontiguousarray(np.asarray(flat, dtype=np.float32).reshape(-1))
        if a.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters, got {a.size}")
        _check(_lib().eptv_unet_set_params(self._h, a.ctypes.data, _stream(stream)), "eptv_unet_set_params")

    def params(self, stream=None):
        import numpy as np
        a = np.zeros(self.n_params, np.float32)
        _check(_lib().eptv_unet_get_params(self._h, a.ctypes.data, _stream(stream)), "eptv_unet_get_params")
        return a

    def grads(self, stream=None):
        import numpy as np
        a = np.zeros(self.n_params, np.float32)
        _check(_lib().eptv_unet_get_grads(self._h, a.ctypes.data, _stream(stream)), "eptv_unet_get_grads")
        return a

    def _act(self, t: torch.Tensor, c: int, name: str) -> torch.Tensor:
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or t.device != self.device:
            raise TypeError(f"{name} must be a float32 tensor on {self.device}")
        if t.dim() != 4 or tuple(t.shape[1:]) != (self.h, self.w, c) or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous [n][{self.h}][{self.w}][{c}], got {tuple(t.shape)}")
        if not 1 <= t.shape[0] <= self.max_batch:
            raise ValueError(f"{name}: batch {t.shape[0]} outside 1..{self.max_batch}")
        return t

    def forward(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        x = self._act(x, self.c_in, "x")
        y = torch.empty((x.shape[0], self.h, self.w, self.c_out), dtype=torch.float32, device=self.device)
        _check(_lib().eptv_unet_forward(self._h, x.data_ptr(), x.shape[0], y.data_ptr(), _stream(stream)),
               "eptv_unet_forward")
        return y

    def backward(self, dy: torch.Tensor, want_dx: bool = False, stream=None):
        dy = self._act(dy, self.c_out, "dy")
        dx = torch.empty((dy.shape[0], self.h, self.w, self.c_in), dtype=torch.float32,
                         device=self.device) if want_dx else None
        _check(_lib().eptv_unet_backward(self._h, dy.data_ptr(), dx.data_ptr() if dx is not None else None,
                                         _stream(stream)), "eptv_unet_backward")
        return dx

    def adam(self, lr: float, step: int, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8,
             stream=None) -> None:
        _check(_lib().eptv_unet_adam(self._h, lr, beta1, beta2, eps, step, _stream(stream)), "eptv_unet_adam")

    def mse(self, y: torch.Tensor, target: torch.Tensor, want_grad: bool = True, stream=None):
        """(loss as a 1-element device tensor, dy or None)."""
        if y.shape != target.shape or not y.is_contiguous() or not target.is_contiguous():
            raise ValueError("y and target must be contiguous and of one shape")
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        dy = torch.empty_like(y) if want_grad else None
        _check(_lib().eptv_unet_mse(self._h, y.data_ptr(), target.data_ptr(), y.numel(),
                                    dy.data_ptr() if dy is not None else None, loss.data_ptr(), _stream(stream)),
               "eptv_unet_mse")
        return loss, dy


def _dev_f32(t, shape, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float32 GPU tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t


def maps_from_eptv(f: torch.Tensor, wx: Optional[torch.Tensor] = None, wy: Optional[torch.Tensor] = None,
                   scale: float = 1.0, f_base: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                   stream=None) -> torch.Tensor:
    """Network tensor [n][ny][nx][3] (wx right, wy above, scale*(f - f_base))
    or, without weights, [n][ny][nx][1], from f [n][ny][nx] (or [ny][nx]);
    written into ``out`` when given."""
    f3 = f if f.dim() == 3 else f.view(1, *f.shape)
    n, ny, nx = f3.shape
    _dev_f32(f3, (n, ny, nx), "f")
    if f_base is not None:
        f_base = _dev_f32(f_base if f_base.dim() == 3 else f_base.view(1, *f_base.shape), (n, ny, nx), "f_base")
    if (wx is None) != (wy is None):
        raise ValueError("give both weight maps or neither")
    c = 1
    if wx is not None:
        wx = _dev_f32(wx if wx.dim() == 3 else wx.view(1, *wx.shape), (n, ny, nx + 1), "wx")
        wy = _dev_f32(wy if wy.dim() == 3 else wy.view(1, *wy.shape), (n, ny + 1, nx), "wy")
        c = 3
    if out is None:
        out = torch.empty((n, ny, nx, c), dtype=torch.float32, device=f.device)
    _dev_f32(out, (n, ny, nx, c), "out")
    _check(_lib().eptv_maps_from_eptv(n, ny, nx, f3.data_ptr(), f_base.data_ptr() if f_base is not None else None,
                                      wx.data_ptr() if wx is not None else None,
                                      wy.data_ptr() if wy is not None else None, scale, out.data_ptr(),
                                      _stream(stream)), "eptv_maps_from_eptv")
    return out


def maps_to_eptv(maps: torch.Tensor, scale: float = 1.0, f_base: Optional[torch.Tensor] = None, stream=None):
    """(f [n][ny][nx], wx [n][ny][nx+1], wy [n][ny+1][nx]) from a 3-channel
    network tensor [n][ny][nx][3]: f = max(channel 2 / scale + f_base, 0)."""
    if maps.dim() != 4 or maps.shape[3] != 3:
        raise ValueError(f"maps must be [n][ny][nx][3], got {tuple(maps.shape)}")
    n, ny, nx, _ = maps.shape
    _dev_f32(maps, (n, ny, nx, 3), "maps")
    if f_base is not None:
        f_base = _dev_f32(f_base if f_base.dim() == 3 else f_base.view(1, *f_base.shape), (n, ny, nx), "f_base")
    f = torch.empty((n, ny, nx), dtype=torch.float32, device=maps.device)
    wx = torch.empty((n, ny, nx + 1), dtype=torch.float32, device=maps.device)
    wy = torch.empty((n, ny + 1, nx), dtype=torch.float32, device=maps.device)
    _check(_lib().eptv_maps_to_eptv(n, ny, nx, maps.data_ptr(), scale,
                                    f_base.data_ptr() if f_base is not None else None, f.data_ptr(), wx.data_ptr(),
                                    wy.data_ptr(), _stream(stream)), "eptv_maps_to_eptv")
    return f, wx, wy
