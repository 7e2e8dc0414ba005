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


def test_server_and_proposal_host_validation_without_gpu():
    """Serving and proposal entry points reject bad arguments before any HIP call."""
    from paper_2606_15476_amd import _lib
    h = ctypes.c_void_p()
    bad_configs = [
        dict(slots=0, max_batch_q=4, max_batch_rel=8, k=10),       # no slot
        dict(slots=65, max_batch_q=4, max_batch_rel=8, k=10),      # too many slots
        dict(slots=1, max_batch_q=0, max_batch_rel=8, k=10),       # empty batch
        dict(slots=1, max_batch_q=2, max_batch_rel=17, k=10),      # more than 8 relations per query
        dict(slots=1, max_batch_q=2, max_batch_rel=4, k=0),        # k < 1
        dict(slots=1, max_batch_q=2, max_batch_rel=4, k=1025),     # k > FARM_MAX_K
    ]
    for c in bad_configs:
        cfg = _lib.ServerConfig(c["slots"], c["max_batch_q"], c["max_batch_rel"], c["k"], 0, 0, 1 << 30)
        assert _lib.L.farm_server_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
        assert b"configuration" in _lib.L.farm_last_error()
    assert _lib.L.farm_server_create(None, ctypes.byref(h)) == -1
    assert _lib.L.farm_server_free(None) == 0
    assert _lib.L.farm_server_progress(None, None, None) == -1
    assert _lib.L.farm_server_cancel(None, 1) == -1
    assert _lib.L.farm_build_proposals(None, None, 8, None) == -1
    stats = (ctypes.c_int64 * 2)()
    assert _lib.L.farm_workspace_proposal_stats(None, stats, 0, None) == -1
