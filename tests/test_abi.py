"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
symbol ksdf.h declares, and its host cell builder agrees with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from paper_2603_29227_amd import ksdf, scenes

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "ksdf.h")
ERR_INVALID_ARGUMENT = -1   # KSDF_ERR_INVALID_ARGUMENT in ksdf.h


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ksdf_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 14
    L = ksdf.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(ksdf.EXPORTS) <= set(names)


@pytest.mark.parametrize("make", [scenes.sphere_workload,
                                  lambda: scenes.small_room_workload(n_queries=8),
                                  lambda: scenes.small_room_workload(n_queries=8, uneven=True)])
def test_host_cell_builder_matches_oracle_bit_exactly(make):
    wl = make()
    c = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min,
                         wl.m_cap_grid, wl.key_lo)
    o = oracle.cells_for(wl)
    np.testing.assert_array_equal(c.offsets, o.offsets)
    np.testing.assert_array_equal(c.samples, o.samples)
    np.testing.assert_array_equal(c.keys, o.keys)


def test_builder_rejects_bad_arguments():
    pts = np.zeros((4, 3), np.float32)
    with pytest.raises(ksdf.KsdfError):
        ksdf.build_cells(pts, (0, 0, 0), -1.0, 0.5, 8, 1)
    with pytest.raises(ksdf.KsdfError):
        ksdf.build_cells(pts, (0, 0, 0), 1.0, 0.5, 500, 1)
    bad = pts.copy()
    bad[2, 1] = np.nan
    with pytest.raises(ksdf.KsdfError, match="non-finite"):
        ksdf.build_cells(bad, (0, 0, 0), 1.0, 0.5, 8, 1)


def test_empty_point_set_gives_no_cells():
    c = ksdf.build_cells(np.zeros((0, 3), np.float64), (0, 0, 0), 1.0, 0.5, 8, 1)
    assert c.n == 0 and c.offsets.tolist() == [0]


def test_status_strings():
    L = ksdf.lib()
    assert L.ksdf_status_string(0) == b"ok"
    assert b"workspace" in L.ksdf_status_string(-3)


def _bytes(cells, wl, flags=0, precision=ksdf.FP32, qbox=None, k_fuse=8):
    L = ksdf.lib()
    hp = ksdf.Hyper(wl.ell, wl.noise_var, -1.0, k_fuse, precision, 1e6, flags, 0)
    off = np.ascontiguousarray(cells.offsets, np.int32)
    smp = np.ascontiguousarray(cells.samples, np.int32)
    keys = np.ascontiguousarray(cells.keys, np.int32)
    lo = hi = None
    if qbox is not None:
        lo, hi = ksdf._d3(qbox[0]), ksdf._d3(qbox[1])
    return L.ksdf_model_bytes(cells.n, off.ctypes.data, smp.ctypes.data, keys.ctypes.data,
                              ksdf._d3(wl.origin), wl.h, len(wl.points), ctypes.byref(hp), lo, hi)


def test_model_bytes_is_a_host_query_that_grows_with_the_options():
    """ksdf_model_bytes sizes the caller-owned store on the host (no device needed):
    the adjoint storage, the var_f storage, the dense inverses (16 KiB per cell) and a
    larger query box each add bytes; invalid arguments give 0."""
    wl = scenes.small_room_workload(n_queries=8)
    c = ksdf.build_cells(wl.points, wl.origin, wl.h, wl.margin, wl.m_max, wl.m_min)
    base = _bytes(c, wl)
    assert base > 0
    adj = _bytes(c, wl, ksdf.FIT_ADJOINT)
    varf = _bytes(c, wl, ksdf.FIT_ADJOINT | ksdf.FIT_ADJOINT_VARF)
    dinv = _bytes(c, wl, ksdf.FIT_DENSE_INV)
    assert base < adj < varf
    assert dinv - base >= 4096 * 4 * c.n
    assert _bytes(c, wl, ksdf.FIT_DENSE_INV, precision=ksdf.FP64) == _bytes(c, wl, precision=ksdf.FP64)
    assert _bytes(c, wl, qbox=((-5, -5, -5), (15, 15, 15))) > base
    assert _bytes(c, wl, k_fuse=99) == 0
    bad = ksdf.CellSet(c.offsets.copy(), c.samples.copy(), c.keys.copy())
    bad.samples[0] = len(wl.points) + 1
    assert _bytes(bad, wl) == 0


def test_query_entry_points_reject_a_null_model_without_a_device():
    """Argument errors are returned before any device work: a null model gives
    KSDF_ERR_INVALID_ARGUMENT from the query calls, also on a host with no GPU."""
    L = ksdf.lib()
    L.ksdf_query_bucket.restype = ctypes.c_int
    L.ksdf_query_bucketed.restype = ctypes.c_int
    assert L.ksdf_query_bucket(None, None, 0, None, 0, None) == ERR_INVALID_ARGUMENT
    assert L.ksdf_query_bucketed(None, None, 0, None, None, None, None, None, None, None, None,
                                 None, 0, None) == ERR_INVALID_ARGUMENT
    assert L.ksdf_query(None, None, 0, None, None, None, None, None, None, None, None, None, 0,
                        None) == ERR_INVALID_ARGUMENT
