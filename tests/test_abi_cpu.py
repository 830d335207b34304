"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/mls.h declares, and rejects bad arguments on the host
before touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mls.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(mls_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2401_03365_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_2401_03365_amd import build
        build.build()
    return _abi.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("mls_build_grid", "mls_project", "mls_project_backward", "mls_knn",
                     "mls_grid_workspace_bytes", "mls_project_workspace_bytes"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2401_03365_amd import _abi
    names = declared_functions()
    assert set(names) == set(_abi.SIGNATURES), "binding and header disagree"
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    from paper_2401_03365_amd import _abi
    for code in range(7):
        assert lib.mls_status_string(code)
    assert b"gfx950" in lib.mls_version()


def test_workspace_sizes(lib):
    assert lib.mls_grid_workspace_bytes(0, 1) == 0
    assert lib.mls_grid_workspace_bytes(10, 0) == 0
    a = lib.mls_grid_workspace_bytes(1000, 1)
    b = lib.mls_grid_workspace_bytes(100000, 1)
    assert 0 < a < b
    assert b >= 100000 * (16 + 4 + 24)  # sorted points, inverse permutation, sort buffers
    assert lib.mls_project_workspace_bytes(None, 32, 10) == 0


def test_build_grid_rejects_bad_arguments_on_host(lib):
    from paper_2401_03365_amd import _abi
    P = ctypes.c_void_p
    h = (ctypes.c_double * 1)(0.1)
    out = P()
    fake = P(0x100000)  # never dereferenced: validation fails first
    ws = lib.mls_grid_workspace_bytes(100, 1)
    # null output handle
    assert lib.mls_build_grid(fake, 100, None, 1, h, None, fake, ws, None, None) == \
        _abi.MLS_ERR_INVALID_ARGUMENT
    # null points
    assert lib.mls_build_grid(None, 100, None, 1, h, None, fake, ws, None, ctypes.byref(out)) == \
        _abi.MLS_ERR_INVALID_ARGUMENT
    # bad h
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        hb = (ctypes.c_double * 1)(bad)
        assert lib.mls_build_grid(fake, 100, None, 1, hb, None, fake, ws, None,
                                  ctypes.byref(out)) == _abi.MLS_ERR_INVALID_ARGUMENT
    # offsets not spanning the points / not ascending
    h2 = (ctypes.c_double * 2)(0.1, 0.1)
    for offs in ((0, 50, 99), (1, 50, 100), (0, 60, 50)):
        o = (ctypes.c_int64 * 3)(*offs)
        assert lib.mls_build_grid(fake, 100, o, 2, h2, None, fake, ws, None,
                                  ctypes.byref(out)) == _abi.MLS_ERR_INVALID_ARGUMENT
    # more than one cloud without offsets
    assert lib.mls_build_grid(fake, 100, None, 2, h2, None, fake, ws, None,
                              ctypes.byref(out)) == _abi.MLS_ERR_INVALID_ARGUMENT
    # misaligned workspace
    assert lib.mls_build_grid(fake, 100, None, 1, h, None, P(0x100010), ws, None,
                              ctypes.byref(out)) == _abi.MLS_ERR_INVALID_ARGUMENT
    # workspace too small
    assert lib.mls_build_grid(fake, 100, None, 1, h, None, fake, ws - 1, None,
                              ctypes.byref(out)) == _abi.MLS_ERR_WORKSPACE_TOO_SMALL
    assert out.value is None


def test_project_rejects_bad_arguments_on_host(lib):
    from paper_2401_03365_amd import _abi
    fake = ctypes.c_void_p(0x100000)
    prm = _abi.MlsParams(k=8, precision=0, support_radius_h=3.0, min_support=3, stages=0)
    # null grid
    assert lib.mls_project(None, ctypes.byref(prm), fake, 0, 10, None, fake, fake, None, fake,
                           1 << 20, None) == _abi.MLS_ERR_INVALID_ARGUMENT
    assert lib.mls_knn(None, 8, fake, 0, 10, None, fake, None, fake, 1 << 20, None) == \
        _abi.MLS_ERR_INVALID_ARGUMENT
    assert lib.mls_project_backward(None, ctypes.byref(prm), fake, 0, 10, None, None, fake, fake,
                                    fake, fake, 1 << 20, None) == _abi.MLS_ERR_INVALID_ARGUMENT
    # null params
    assert lib.mls_project(None, None, fake, 0, 10, None, fake, fake, None, fake, 1 << 20,
                           None) == _abi.MLS_ERR_INVALID_ARGUMENT
    assert lib.mls_grid_destroy(None) == _abi.MLS_ERR_INVALID_ARGUMENT


def test_grid_entry_points_reject_a_null_grid(lib):
    # every call that takes a grid handle refuses a null one on the host,
    # before anything is launched (no device is needed to see the code)
    from paper_2401_03365_amd import _abi
    P = ctypes.c_void_p
    fake = P(0x100000)
    bad = _abi.MLS_ERR_INVALID_ARGUMENT
    prm = _abi.MlsParams(k=8, precision=0, support_radius_h=3.0, min_support=3, stages=0)
    info = _abi.MlsGridInfo()
    origin, cell = (ctypes.c_double * 3)(), ctypes.c_double()
    dims = (ctypes.c_int32 * 3)()
    p1, p2, p3 = P(), P(), P()
    cap = ctypes.c_int64()
    assert lib.mls_rebuild_grid(None, fake, None) == bad
    assert lib.mls_get_grid_info(None, ctypes.byref(info)) == bad
    assert lib.mls_get_cloud_grid(None, 0, origin, ctypes.byref(cell), dims) == bad
    assert lib.mls_grid_sorted_points(None, ctypes.byref(p1), ctypes.byref(p2)) == bad
    assert lib.mls_grid_cell_table(None, ctypes.byref(p1), ctypes.byref(cap),
                                   ctypes.byref(p3)) == bad
    assert lib.mls_project_geometry(None, ctypes.byref(prm), fake, 0, 10, None, fake, fake,
                                    None, fake, fake, fake, 1 << 20, None) == bad
    assert lib.mls_project_noalloc(None, ctypes.byref(prm), fake, 0, 10, None, fake, fake,
                                   None, None) == bad
    assert lib.mls_project_backward_workspace_bytes(None, 8, 10, 0) == 0
    # and the tuner refuses null inputs the same way
    h = (ctypes.c_double * 1)(0.1)
    cand = (ctypes.c_double * 2)(1.0, 1.25)
    best = ctypes.c_double()
    assert lib.mls_autotune_cell(None, 100, None, 1, h, 8, cand, 2, 1, fake, 1 << 20, None,
                                 ctypes.byref(best), None) == bad
    assert lib.mls_autotune_workspace_bytes(0, 1, 8, 1) == 0


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_2401_03365_amd import _abi
    with pytest.raises(RuntimeError, match="not found"):
        _abi._lib_backup = _abi._lib
        try:
            _abi._lib = None
            _abi.load(str(tmp_path / "missing.so"))
        finally:
            _abi._lib = _abi._lib_backup
