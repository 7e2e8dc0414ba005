"""CPU-side checks of the C-ABI library: it loads and exports every entry
point the public header declares (no compute calls -- there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "farm.h")


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"FARM_API\s+[\w\s\*]+?\b(farm_\w+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared_functions()
    for required in ("farm_build_memory", "farm_score_query", "farm_topk", "farm_query_topk"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2606_15476_amd import _lib
    lib = ctypes.CDLL(_lib.lib_path())
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"libfarm.so lacks {missing}"
    assert set(_lib.EXPORTS) == set(declared_functions())


def test_version_and_error_strings_without_gpu():
    from paper_2606_15476_amd import _lib
    assert b"gfx950" in _lib.L.farm_version()
    assert _lib.L.farm_last_error() is not None


def test_host_validation_rejects_bad_arguments_without_touching_the_gpu():
    """Argument checks that happen before any HIP call."""
    from paper_2606_15476_amd import _lib
    h = ctypes.c_void_p()
    # n = 0
    assert _lib.L.farm_build_memory(0, 4, None, None, None, None, None, 1.0, 0.0, 0, None, ctypes.byref(h)) == -1
    assert b"n = 0" in _lib.L.farm_last_error()
    # d out of range
    assert _lib.L.farm_build_memory(5, 0, None, None, None, None, None, 1.0, 0.0, 0, None, ctypes.byref(h)) == -1
    # null workspace / memory
    assert _lib.L.farm_score_query(None, None, 1, 4, None, None, None, None, None, None, None, None, None) == -1
    assert _lib.L.farm_workspace_create(None, 1, 1, 10, ctypes.byref(h)) == -1
    assert _lib.L.farm_free_memory(None) == 0
