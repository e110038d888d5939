"""The C-ABI library loads and exports every symbol include/sampx.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os

import pytest

from paper_2301_04835_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.load()


def test_header_declares_the_boundary():
    names = _lib.header_symbols()
    for required in ["sx_create", "sx_destroy", "sx_add_cv_dihedral", "sx_add_cv_gyration",
                     "sx_add_cv_coordination", "sx_metad_config", "sx_abf_config", "sx_set_walkers",
                     "sx_state_bytes", "sx_workspace_bytes", "sx_bind", "sx_step", "sx_eval_cv", "sx_cv_vjp",
                     "sx_hillsum", "sx_deposit", "sx_hills_set", "sx_hills_get", "sx_abf_grid_get",
                     "sx_state_export", "sx_state_import", "sx_graph_capture", "sx_graph_launch", "sx_autotune"]:
        assert required in names
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in _lib.header_symbols() if not hasattr(lib, n)]
    assert not missing


def test_measurement_library_exports_its_header(lib):
    """include/sampx_measure.h: the sxm_* hooks come from libsampx.so, the
    timing and probe calls from libsampx_measure.so; the binding knows each."""
    names = _lib.header_symbols(_lib.MEASURE_HEADER)
    names = [n for n in names if n not in _lib.header_symbols()]
    assert set(names) == set(_lib.MEASURE_HOOKS) | set(_lib.MEASURE_SIGNATURES)
    assert all(hasattr(lib, n) for n in _lib.MEASURE_HOOKS)
    M = _lib.load_measure()
    assert all(hasattr(M, n) for n in _lib.MEASURE_SIGNATURES)
    # the measurement calls are not part of the biasing-path boundary
    assert not set(_lib.MEASURE_SIGNATURES) & set(_lib.header_symbols())


def test_status_strings_and_null_handling(lib):
    assert lib.sx_status_string(0) == b"ok"
    assert lib.sx_status_string(3) == b"hill capacity exceeded"
    assert lib.sx_status_string(99) == b"unknown status"
    assert lib.sx_create(None, 0, None) == _lib.SX_EINVAL
    assert lib.sx_num_cvs(None) == 0
    lib.sx_destroy(None)  # ignored


def test_create_without_device_reports_device_error(lib):
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is visible")
    except Exception:
        pass
    h = ctypes.c_void_p()
    assert lib.sx_create(ctypes.byref(h), 0, None) == _lib.SX_EDEVICE
    assert not h.value
