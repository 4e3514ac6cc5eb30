"""The float32 system matrix the HIP kernels evaluate, computed on the host by
the library itself (eptv_geometry_matrix, no GPU), against the FP64 oracle's
Siddon matrix entry by entry.  CPU only."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1009_2288_amd import synth
from paper_1009_2288_amd.synth import Geometry, fan_dbeta

GEOMS = {
    "small": synth.geometry_small,
    "ragged": lambda: Geometry(77, 53, 1.1, 13, 101, fan_dbeta(77, 53, 1.1, 150.0, 101) * 1.05, 150.0, 300.0, 0.3),
    "odd": lambda: Geometry(65, 65, 1.0, 7, 129, fan_dbeta(65, 65, 1.0, 120.0, 129), 120.0, 240.0),
    "gridline": lambda: Geometry(16, 16, 1.0, 1, 9, fan_dbeta(16, 16, 1.0, 60.0, 9), 60.0, 120.0, 0.0, np.array([0.0])),
    "paper": synth.geometry_paper,
}


def as_sparse(rp, col, val, shape):
    return sp.csr_matrix((np.asarray(val, np.float64), np.asarray(col), np.asarray(rp)), shape=shape)


@pytest.mark.parametrize("name", list(GEOMS))
def test_kernel_matrix_matches_oracle_entrywise(oracle, name):
    from paper_1009_2288_amd import eptv
    g = GEOMS[name]()
    shape = (g.n_views * g.n_bins, g.nx * g.ny)
    A32 = as_sparse(*eptv.geometry_matrix(g), shape)
    A64 = as_sparse(*oracle.Matrix(g).csr(), shape)
    D = (A32 - A64).tocoo()
    # Each float32 entry is the exact chord up to (i) two float roundings
    # (<= 3e-7 relative) and (ii) the 32.32 fixed-point position of the ray,
    # <= (nx + ny) 2^-32 rows, which moves length between the two pixels of a
    # row crossing in proportion to the length per row crossed, d / |minor
    # direction component|.
    th = g.angles()[:, None]
    beta = (np.arange(g.n_bins)[None, :] - 0.5 * (g.n_bins - 1) + g.bin_offset) * g.dbeta_rad
    minor = np.minimum(np.abs(np.cos(th + beta)), np.abs(np.sin(th + beta))).ravel()
    w = g.pixel_mm / np.maximum(minor, 1e-300)
    ref = np.asarray(abs(A64)[D.row, D.col]).ravel()
    bound = 3e-7 * ref + (g.nx + g.ny) * 2.0 ** -32 * w[D.row] + 1e-12
    assert np.all(np.abs(D.data) <= bound)
    # per ray the total length agrees to float rounding
    rs32, rs64 = np.asarray(A32.sum(1)).ravel(), np.asarray(A64.sum(1)).ravel()
    assert np.all(np.abs(rs32 - rs64) <= 3e-7 * rs64 + 1e-9)
    # the same pattern, apart from slivers of a corner far below float resolution
    only32 = (A32 != 0).astype(int) - (A64 != 0).astype(int)
    extra = abs(only32).sum()
    assert extra <= 1e-5 * A64.nnz + 2


def test_kernel_matrix_rows_are_sweep_ordered(oracle):
    from paper_1009_2288_amd import eptv
    g = GEOMS["small"]()
    rp, col, val = eptv.geometry_matrix(g)
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == col.size
    assert np.all(val > 0) and col.min() >= 0 and col.max() < g.nx * g.ny
    # entries follow the sweep: along a ray the sweep index (column, or row for
    # rays closer to the y axis) never decreases and steps by at most one
    for r in range(0, g.n_views * g.n_bins, 97):
        c = col[rp[r]:rp[r + 1]]
        i, j = c % g.nx, c // g.nx
        di, dj = np.diff(i), np.diff(j)
        assert (np.all((di >= 0) & (di <= 1)) and np.all(np.abs(dj) <= 2)) or \
               (np.all((dj >= 0) & (dj <= 1)) and np.all(np.abs(di) <= 2))
