"""The C ABI library loads, exports every function declared in include/boac.h, and validates its
arguments before touching the device (these tests make no compute call and run without a GPU)."""
import ctypes

import pytest

from paper_2109_11920_amd import _lib
from paper_2109_11920_amd._lib import BoacGeom, BoacSlice


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_header_declares_the_documented_entry_points():
    names = _lib.header_functions()
    for required in ("boac_rasterize_mu", "boac_project", "boac_backproject", "boac_mlem", "boac_objective",
                     "boac_objective_grad", "boac_evaluate_batch", "boac_ctx_create", "boac_ctx_destroy",
                     "boac_last_error"):
        assert required in names


def test_library_exports_every_header_symbol(lib):
    for name in _lib.header_functions():
        assert hasattr(lib, name), name
    assert set(_lib.header_functions()) == set(_lib._SIGNATURES)


def test_version(lib):
    v = lib.boac_version()
    assert v >> 16 == 1


def _good():
    return BoacGeom(64, 64, 64, 64, 0.4)


ALIGNED = ctypes.c_void_p(1 << 20)       # never dereferenced: validation fails before any launch
MISALIGNED = ctypes.c_void_p((1 << 20) + 4)


@pytest.mark.parametrize("field,value", [("n", 1), ("n", 2000), ("n_angles", 1), ("n_bins", 0),
                                         ("n_samples", 5000), ("pixel_cm", 0.0), ("pixel_cm", float("nan")),
                                         ("n_bins", 400)])
def test_bad_geometry_is_rejected_before_the_device(lib, field, value):
    g = _good()
    setattr(g, field, value)
    st = lib.boac_project(None, ctypes.byref(g), ALIGNED, ALIGNED, 1, ALIGNED, None)
    assert st == 2, lib.boac_last_error()
    assert lib.boac_last_error()


def test_bad_counts_and_pointers(lib):
    g = _good()
    assert lib.boac_project(None, ctypes.byref(g), ALIGNED, ALIGNED, 0, ALIGNED, None) == 1
    assert lib.boac_project(None, ctypes.byref(g), None, ALIGNED, 1, ALIGNED, None) == 1
    assert b"NULL" in lib.boac_last_error()
    assert lib.boac_project(None, ctypes.byref(g), MISALIGNED, ALIGNED, 1, ALIGNED, None) == 1
    assert b"aligned" in lib.boac_last_error()
    assert lib.boac_mlem(None, ctypes.byref(g), ALIGNED, ALIGNED, 1, -1, ALIGNED, None) == 1
    assert lib.boac_objective(None, ctypes.byref(g), ALIGNED, ALIGNED, 1, 0.0, 5, ALIGNED, None, None, None) == 1
    assert lib.boac_objective_grad(None, ctypes.byref(g), ALIGNED, ALIGNED, 1, 0.8, 5, 0, ALIGNED, ALIGNED,
                                   None, None) == 1
    assert lib.boac_rasterize_mu(None, None, ALIGNED, 1, 0.8, ALIGNED, None) == 1
    assert lib.boac_objective_grad_ex(None, ctypes.byref(g), ALIGNED, ALIGNED, 1, 0.8, 5, 5, 2, ALIGNED, ALIGNED,
                                      None, None) == 1
    assert b"grad_mode" in lib.boac_last_error()
    assert lib.boac_objective_grad_ex(None, ctypes.byref(g), ALIGNED, ALIGNED, 1, 0.8, 5, 5, 1, ALIGNED, None,
                                      None, None) == 1


def test_null_context_after_valid_arguments(lib):
    g = _good()
    st = lib.boac_project(None, ctypes.byref(g), ALIGNED, ALIGNED, 1, ALIGNED, None)
    assert st == 1 and b"context" in lib.boac_last_error()


def test_batch_validation(lib):
    arr = (BoacSlice * 2)()
    arr[0] = BoacSlice(_good(), ALIGNED, ALIGNED, 4, ALIGNED, None, None)
    arr[1] = BoacSlice(BoacGeom(64, 64, 64, 64, -1.0), ALIGNED, ALIGNED, 4, ALIGNED, None, None)
    assert lib.boac_evaluate_batch(None, arr, 2, 0.8, 10, 5, None) == 2
    assert b"slice 1" in lib.boac_last_error()
    assert lib.boac_evaluate_batch(None, arr, 0, 0.8, 10, 5, None) == 1
    assert lib.boac_evaluate_batch(None, None, 1, 0.8, 10, 5, None) == 1


def test_stats_need_a_context(lib):
    assert lib.boac_ctx_set_profiling(None, 1) == 1
    assert lib.boac_ctx_reset_stats(None) == 1
    lib.boac_ctx_destroy(None)  # no-op


def test_gp_entry_points_validate_before_the_device(lib):
    from paper_2109_11920_amd._lib import BoacGpInfo
    info = BoacGpInfo(4, 8, 0.5, 1.0, 1e-6, 10.0, 2.0, -3.0)
    args = lambda M, best=1.0, xi=0.0: (None, ctypes.byref(info), ALIGNED, ALIGNED, ALIGNED, ALIGNED, M, best, xi,
                                        None, None, ALIGNED, None)
    assert lib.boac_gp_ei(*args(0)) == 1 and b"M" in lib.boac_last_error()
    assert lib.boac_gp_ei(*args((1 << 20) + 1)) == 1
    assert lib.boac_gp_ei(*args(16, xi=-1.0)) == 1
    assert lib.boac_gp_ei(*args(16, best=float("inf"))) == 1
    bad = BoacGpInfo(4, 8, 0.0, 1.0, 1e-6, 10.0, 2.0, -3.0)
    assert lib.boac_gp_ei(None, ctypes.byref(bad), ALIGNED, ALIGNED, ALIGNED, ALIGNED, 16, 1.0, 0.0, None, None,
                          ALIGNED, None) == 1
    assert lib.boac_gp_ei(None, None, ALIGNED, ALIGNED, ALIGNED, ALIGNED, 16, 1.0, 0.0, None, None, ALIGNED,
                          None) == 1
    # valid arguments, no context: refused before any device call
    assert lib.boac_gp_ei(*args(16)) == 1 and b"context" in lib.boac_last_error()
    assert lib.boac_gp_fit(None, None, 0, 8, None, 1, 0, 1e-6, None, None, None) == 1



def test_noalloc_rejects_a_geometry_beyond_its_scratch_before_the_device(lib):
    # 1024 x 1024, 512 angles: one candidate's attenuation tensor alone is 2 GB, beyond the fixed array
    g = BoacGeom(1024, 512, 1024, 1024, 0.025)
    st = lib.boac_objective_noalloc(None, ctypes.byref(g), ALIGNED, ALIGNED, 1, 0.8, 5, ALIGNED, None, None, None)
    assert st == 3 and b"no-allocation scratch" in lib.boac_last_error()
    # valid sizes, no context: refused before any device call
    st = lib.boac_objective_noalloc(None, ctypes.byref(_good()), ALIGNED, ALIGNED, 4, 0.8, 5, ALIGNED, None, None,
                                    None)
    assert st == 1 and b"context" in lib.boac_last_error()


def test_device_search_entry_point_validates_before_the_device(lib):
    from paper_2109_11920_amd._lib import BoacGpInfo
    info = BoacGpInfo(4, 8, 0.5, 1.0, 1e-6, 10.0, 2.0, -3.0)

    def call(P, nc, n_local=3, r0=0.1, shrink=0.85):
        return lib.boac_gp_chaos_local(None, ctypes.byref(info), ALIGNED, ALIGNED, ALIGNED, 1.0, 0.0, ALIGNED, P,
                                       ALIGNED, ALIGNED, nc, r0, shrink, n_local, ALIGNED, ALIGNED, None)
    assert call(4, 5) == 1 and b"n_centres" in lib.boac_last_error()
    assert call(0, 1) == 1
    assert call(64, 8, n_local=-1) == 1
    assert call(64, 8, r0=float("nan")) == 1
    assert call(64, 8, shrink=-0.5) == 1
    assert call((1 << 21), 1) == 1 and b"M" in lib.boac_last_error()   # per x n_centres above 2^20
    # valid arguments, no context: refused before any device call
    assert call(64, 8) == 1 and b"context" in lib.boac_last_error()


def test_device_whole_search_validates_before_the_device(lib):
    from paper_2109_11920_amd._lib import BoacGpInfo
    info = BoacGpInfo(4, 8, 0.5, 1.0, 1e-6, 10.0, 2.0, -3.0)
    cnt, mx, nq = ctypes.c_int32(), ctypes.c_double(), ctypes.c_int64()

    def call(P=512, ng=4, nl=4, centres=8, q=8, r0=0.1, shrink=0.85, excl=0.02, per=64, T=0, taken=None,
             props=ALIGNED, counts=True):
        return lib.boac_gp_chaos_search(None, ctypes.byref(info), ALIGNED, ALIGNED, ALIGNED, 1.0, 0.0, ALIGNED, P, ng,
                                        nl, centres, q, r0, shrink, excl, per, taken, T, props,
                                        ctypes.byref(cnt) if counts else None, ctypes.byref(mx), ctypes.byref(nq),
                                        None)
    assert call(P=0) == 1 and b"chains" in lib.boac_last_error()
    assert call(P=8193) == 1
    assert call(ng=0) == 1 and call(nl=-1) == 1
    assert call(q=0) == 1 and call(per=0) == 1 and call(centres=0) == 1
    assert call(excl=-1.0) == 1 and call(r0=float("inf")) == 1
    assert call(P=4096, ng=8, nl=8, per=4096) == 1 and b"pool" in lib.boac_last_error()
    assert call(T=3) == 1   # taken rows without a pointer
    assert call(counts=False) == 1
    # valid arguments, no context: refused before any device call
    assert call() == 1 and b"context" in lib.boac_last_error()
