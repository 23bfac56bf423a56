"""The C ABI library loads and exports every function declared in include/lp.h;
argument validation that happens before any device call (no GPU needed)."""

from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "lp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    names = header_functions()
    for n in ("fieldset_create", "fieldset_push_snapshot", "pset_create", "pset_execute",
              "pset_status", "pset_get", "pset_records", "lp_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1707_05163_amd import _lib
    lib = C.CDLL(_lib.LIBPATH)
    for n in header_functions():
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTS) == header_functions()


def test_validation_before_device_work():
    from paper_1707_05163_amd import _lib as L
    h = C.c_void_p()
    x = np.arange(4.0)
    bad = np.array([0.0, 1.0, 1.0, 2.0])
    cases = [
        L.lp_grid_desc(1, 4, 0, x.ctypes.data, x.ctypes.data, None, 0, 1, 3, 0.0, None),
        L.lp_grid_desc(4, 4, 1, x.ctypes.data, x.ctypes.data, None, 0, 1, 3, 0.0, None),
        L.lp_grid_desc(4, 4, 0, bad.ctypes.data, x.ctypes.data, None, 0, 1, 3, 0.0, None),
        L.lp_grid_desc(4, 4, 0, x.ctypes.data, x.ctypes.data, None, 0, 9, 3, 0.0, None),
        L.lp_grid_desc(4, 4, 0, x.ctypes.data, x.ctypes.data, None, 0, 1, 0, 0.0, None),
        L.lp_grid_desc(4, 4, 3, x.ctypes.data, x.ctypes.data, None, 0, 1, 3, 0.0, None),
    ]
    for g in cases:
        assert L.lib.fieldset_create(C.byref(g), C.byref(h)) == L.LP_EINVAL
        assert L.lib.lp_last_error()
    o = L.lp_exec_opts()
    assert L.lib.pset_execute(None, 1.0, 1.0, 0.0, C.byref(o), None) == L.LP_EINVAL
    assert L.lib.lp_version().startswith(b"lp-mi355x")


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    import importlib
    from paper_1707_05163_amd import _lib
    monkeypatch.setattr(_lib, "LIBPATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        _lib.load()
    importlib.reload(_lib)
