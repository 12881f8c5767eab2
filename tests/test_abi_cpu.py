"""The C-ABI library loads and exports every symbol the public header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "vdmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vdmc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = _declared_symbols()
    for must in ["vdmc_build_graph", "vdmc_count", "vdmc_count34", "vdmc_count_batch", "vdmc_tune",
                 "vdmc_serve_create", "vdmc_serve_submit", "vdmc_serve_poll", "vdmc_serve_wait",
                 "vdmc_serve_stats", "vdmc_serve_destroy", "vdmc_free_graph", "vdmc_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2201_11655_amd import vdmc
    lib = vdmc.load()
    missing = [s for s in _declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(vdmc.SYMBOLS) == _declared_symbols()


def test_host_only_calls():
    from paper_2201_11655_amd import vdmc
    assert vdmc.num_classes(3) == 13
    assert vdmc.num_classes(4) == 199
    assert vdmc.num_classes(5) == 9364
    assert vdmc.num_classes(2) == -1 and vdmc.num_classes(6) == -1
    lib = vdmc.load()
    assert lib.vdmc_count_supported(None, 5) == -1   # NULL graph
    assert lib.vdmc_class_codes_u32(6, None) == 1 and lib.vdmc_class_table_u16(5, None) == 1
    assert lib.vdmc_free_graph(None) == 0          # NULL is a no-op
    assert lib.vdmc_graph_info(None, None, None, None, None) == 1
    assert b"NULL" in lib.vdmc_last_error()


def test_build_graph_rejects_bad_sizes_before_touching_the_device():
    from paper_2201_11655_amd import vdmc
    lib = vdmc.load()
    h = ctypes.c_void_p()
    assert lib.vdmc_build_graph(-1, 0, None, None, 0, None, ctypes.byref(h)) == 1
    assert lib.vdmc_build_graph(1 << 30, 0, None, None, 0, None, ctypes.byref(h)) == 1
    assert lib.vdmc_build_graph(5, 3, None, None, 0, None, ctypes.byref(h)) == 1
    assert lib.vdmc_build_graph(5, 0, None, None, 0, None, None) == 1


def test_serve_config_validation_without_device():
    """Bad server configurations are rejected before any device call."""
    from paper_2201_11655_amd import vdmc
    lib = vdmc.load()
    h = ctypes.c_void_p()
    assert lib.vdmc_serve_create(None, ctypes.byref(h)) == 1
    cfg = vdmc.ServeConfig(0, 4)
    assert lib.vdmc_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == 1
    cfg = vdmc.ServeConfig(1 << 20, 0)
    assert lib.vdmc_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == 1
    assert lib.vdmc_serve_destroy(None) == 0
    assert lib.vdmc_serve_poll(None, 1, None) == 1
    assert lib.vdmc_count_batch(None, 1, 4, None, None) == 1   # NULL arrays
    assert lib.vdmc_count_batch(None, 0, 6, None, None) == 1   # bad k
    assert lib.vdmc_count_batch(None, 0, 5, None, None) == 0   # k = 5, empty batch
