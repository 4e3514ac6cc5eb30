"""The C-ABI library: it loads, exports every symbol the header declares, and
rejects bad geometry before touching the GPU.  CPU only (no compute calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "eptv.h")


def declared_symbols():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(eptv_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1009_2288_amd import eptv
    return eptv.library()


def test_header_declares_the_path(lib):
    syms = declared_symbols()
    for name in ("eptv_project", "eptv_backproject", "eptv_tv_step", "eptv_reconstruct", "eptv_tv_gradient",
                 "eptv_select_sigma", "eptv_plan_create", "eptv_workspace_bytes"):
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_binding_symbol_list_matches_header():
    from paper_1009_2288_amd import eptv
    assert sorted(eptv.SYMBOLS) == declared_symbols()


def test_status_strings(lib):
    from paper_1009_2288_amd import eptv
    assert lib.eptv_status_string(eptv.EPTV_OK) == b"ok"
    assert lib.eptv_status_string(eptv.EPTV_ERR_GEOMETRY) == b"invalid geometry"
    assert lib.eptv_status_string(99) == b"unknown status"


@pytest.mark.parametrize("field,value,status", [
    ("sad_mm", 50.0, 2),        # source inside the circle through the image corners
    ("dbeta_rad", 0.0, 2),
    ("dbeta_rad", 0.02, 2),     # 256 bins x 0.02 rad: the fan would exceed 180 degrees
    ("pixel_mm", -1.0, 2),
    ("nx", 0, 1),
    ("ny", 1, 1),               # a one-pixel-high image (the projector reads pixel pairs)
    ("n_bins", -3, 1),
    ("nx", 32769, 1),           # beyond the largest image side (32768)
    ("n_views", 5_000_000, 1),  # 1.28e9 rays: beyond the 2^30 limit on views x bins
    ("sdd_mm", 100.0, 2),       # detector closer than the source distance
])
def test_plan_create_rejects_bad_geometry_without_gpu(lib, field, value, status):
    from paper_1009_2288_amd import eptv
    g = dict(nx=128, ny=128, pixel_mm=1.0, n_views=30, view_angles_rad=None, n_bins=256, dbeta_rad=1.42e-3,
             bin_offset=0.0, sad_mm=500.0, sdd_mm=1000.0)
    g[field] = value
    cg = eptv._Geometry(**g)
    h = C.c_void_p()
    assert lib.eptv_plan_create(C.byref(cg), C.byref(h)) == status
    assert not h.value


def test_null_arguments_are_rejected(lib):
    assert lib.eptv_plan_create(None, None) == 1
    assert lib.eptv_plan_destroy(None) == 1
    assert lib.eptv_project(None, None, None, 1.0, 0.0, None, 0, None) == 1
    assert lib.eptv_reconstruct(None, None, None, None, None, None, 0, None, None) == 1


def test_batch_cases_shapes_are_seeded_and_in_range():
    from paper_1009_2288_amd import synth
    a = synth.batch_cases(5, 2, with_phantom=False)
    b = synth.batch_cases(5, 2, with_phantom=False)
    for x, y in zip(a, b):
        assert x.geom == y.geom and np.array_equal(x.y, y.y)
        assert x.geom.nx in (256, 384, 512) and 20 <= x.geom.n_views <= 60 and 368 <= x.geom.n_bins <= 736
        assert 1e4 <= x.i0 <= 1e5 and x.phantom is None


def test_batch_create_rejects_bad_input_without_gpu(lib):
    out = C.c_void_p()
    assert lib.eptv_batch_create(None, 1, C.byref(out)) == 1
    assert lib.eptv_batch_destroy(None) == 1


def test_network_entry_points_reject_bad_input_without_gpu(lib):
    """The U-Net and tensor-conversion calls check their arguments before any
    HIP call: impossible shapes, a missing output, non-positive scales."""
    out = C.c_void_p()
    # channels, base, levels, batch, sizes; height/width must divide by 2^(levels-1)
    assert lib.eptv_unet_create(0, 3, 32, 4, 1, 512, 512, C.byref(out)) == 1
    assert lib.eptv_unet_create(1, 3, 32, 0, 1, 512, 512, C.byref(out)) == 1
    assert lib.eptv_unet_create(1, 3, 32, 4, 0, 512, 512, C.byref(out)) == 1
    assert lib.eptv_unet_create(1, 3, 32, 4, 1, 100, 512, C.byref(out)) == 1
    assert lib.eptv_unet_create(1, 3, 12, 4, 1, 512, 512, C.byref(out)) == 1   # base not a multiple of 8
    assert lib.eptv_unet_create(1, 3, 32, 4, 1, 512, 512, None) == 1
    assert not out.value
    assert lib.eptv_unet_destroy(None) == 1
    n = C.c_longlong()
    assert lib.eptv_unet_param_count(None, C.byref(n)) == 1
    assert lib.eptv_unet_forward(None, None, 1, None, None) == 1
    assert lib.eptv_unet_backward(None, None, None, None) == 1
    assert lib.eptv_unet_adam(None, 1e-3, 0.9, 0.999, 1e-8, 1, None) == 1
    assert lib.eptv_unet_mse(None, None, None, 0, None, None, None) == 1
    fake = C.c_void_p(16)  # never dereferenced: the checks fail first
    assert lib.eptv_maps_from_eptv(0, 4, 4, fake, None, None, None, 1.0, fake, None) == 1
    assert lib.eptv_maps_from_eptv(1, 4, 4, fake, None, fake, None, 1.0, fake, None) == 1  # one weight map only
    assert lib.eptv_maps_from_eptv(1, 4, 4, fake, None, None, None, 0.0, fake, None) == 1
    assert lib.eptv_maps_from_eptv(1, 4, 4, fake, None, None, None, float("inf"), fake, None) == 1
    assert lib.eptv_maps_to_eptv(1, 4, 4, fake, -1.0, None, fake, fake, fake, None) == 1
    assert lib.eptv_maps_to_eptv(1, 4, 4, fake, 1.0, None, fake, None, fake, None) == 1
    assert lib.eptv_reconstruct_weighted(None, None, None, None, None, None, None, 0, None, 0, None, None) == 1


def test_p2_calls_reject_an_eps_whose_square_is_not_normal(lib):
    """The P2 calls divide by the half-edge magnitudes, which eps bounds below:
    eps <= 0, NaN, or an eps whose float square is zero or subnormal is
    rejected before any device call (a fake plan handle is never touched)."""
    from paper_1009_2288_amd import eptv
    fake = C.c_void_p(16)
    n = C.c_size_t()
    for bad in (0.0, -1e-4, 1e-30, 1e-20, float("nan"), float("inf")):
        prm = eptv.Params(tv_eps=bad)._c()
        assert lib.eptv_workspace_bytes(fake, C.byref(prm), C.byref(n)) == 1, bad
        assert lib.eptv_tv_step(fake, C.byref(prm), fake, fake, -1.0, 1, fake, 1 << 20, None, None) == 1, bad
        assert lib.eptv_tv_gradient(fake, fake, fake, 1000.0, 0.01, bad, fake, None, None, fake, 1 << 20,
                                    None) == 1, bad
        assert lib.eptv_tv_gradient_vjp(fake, fake, fake, 1000.0, 0.01, bad, fake, fake, 1 << 20, None) == 1, bad


def test_nonfinite_status_and_params_layout(lib):
    from paper_1009_2288_amd import eptv
    assert lib.eptv_status_string(eptv.EPTV_ERR_NONFINITE) == b"non-finite input"
    # the check flag must be 0 or 1; checked before the plan is touched
    fake = C.c_void_p(16)
    n = C.c_size_t()
    prm = eptv.Params(check_finite=2)._c()
    assert lib.eptv_workspace_bytes(fake, C.byref(prm), C.byref(n)) == 1
    # the binding's structs end with the header's last fields
    src = open(HEADER).read()
    assert src.index("int check_finite;") > src.index("double stop_rmse;")
    assert [f[0] for f in eptv._Params._fields_][-1] == "check_finite"
    assert [f[0] for f in eptv._Stats._fields_][-4:] == ["armijo_q0", "armijo_q1", "cgls_gamma", "cgls_delta"]


def test_stream_read_rejects_bad_arguments_without_gpu(lib):
    """The measurement aid checks its arguments before any HIP call."""
    from paper_1009_2288_amd import eptv
    fn = lib.eptv_stream_read
    buf = C.c_void_p(16 * 1024)  # never dereferenced: every call below is rejected first
    sink = C.c_void_p(64)
    assert fn(None, 1024, sink, None) == eptv.EPTV_ERR_ARG
    assert fn(buf, 1024, None, None) == eptv.EPTV_ERR_ARG
    assert fn(buf, 0, sink, None) == eptv.EPTV_ERR_ARG
    assert fn(buf, 1000, sink, None) == eptv.EPTV_ERR_ARG          # not a multiple of 16 bytes
    assert fn(C.c_void_p(16 * 1024 + 4), 1024, sink, None) == eptv.EPTV_ERR_ARG  # misaligned
