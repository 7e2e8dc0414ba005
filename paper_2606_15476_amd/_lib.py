"""ctypes declarations of libfarm.so (include/farm.h).  Loads the in-tree
library built by ``python -m paper_2606_15476_amd.build``; raises if absent."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
_PATH = os.path.join(_HERE, "libfarm.so")

FARM_OK, FARM_ERR_INVALID_ARG, FARM_ERR_OOM, FARM_ERR_HIP, FARM_ERR_UNSUPPORTED, FARM_ERR_BUSY = 0, -1, -2, -3, -4, -5
F32, BF16, FP8_E4M3 = 0, 1, 2
EXHAUSTIVE, BOUNDED, PROPOSAL = 0, 1, 2
OPT_GLOBAL_PROPOSAL_PASS = 1
NEAR, ABOVE, BELOW, LEFT_OF, RIGHT_OF = 0, 1, 2, 3, 4
NEXT_TO, IN_FRONT_OF, BEHIND, ON = 5, 6, 7, 8
CLOSEST, FARTHEST, INSIDE = 9, 10, 11
BETWEEN, AND = 12, 13  # ternary Between's slot and the slot of its second anchor
# over entity Gaussians (Hellinger Near) and stored views (farm_set_entity_geometry)
NEAR_HELLINGER, LEFT_OF_VIEW, RIGHT_OF_VIEW, IN_FRONT_OF_VIEW, BEHIND_VIEW = 14, 15, 16, 17, 18
NUM_PRED, NUM_PROP_PRED = 19, 9  # predicate ids; those with learned anchor lists
FARM_MAX_REL = 8
FARM_MAX_K = 1024
FARM_NO_ID = 0xFFFFFFFF
FARM_BUILD_BF16, FARM_BUILD_FP8 = 0x1, 0x2

EXPORTS = (
    "farm_build_memory", "farm_set_entity_geometry", "farm_add_embedding_space", "farm_rrf_similarity",
    "farm_query_topk_rrf", "farm_free_memory", "farm_memory_info", "farm_workspace_create", "farm_workspace_free",
    "farm_workspace_bytes", "farm_workspace_estimate", "farm_score_query", "farm_similarity", "farm_topk", "farm_query_topk", "farm_query_topk_static",
    "farm_workspace_status", "farm_last_error", "farm_version", "farm_workspace_set_timing",
    "farm_workspace_timings", "farm_mlp_create", "farm_mlp_free", "farm_mlp_shape", "farm_mlp_get_weights",
    "farm_mlp_get_grads", "farm_mlp_get_batch", "farm_mlp_set_weights", "farm_mlp_table_logits", "farm_mlp_inputs", "farm_mlp_logits", "farm_mlp_step",
    "farm_build_proposals", "farm_build_proposals_by_value", "farm_workspace_proposal_stats", "farm_get_proposals", "farm_proposal_pass_form",
    "farm_server_create", "farm_server_add_scene", "farm_server_submit", "farm_server_cancel", "farm_server_progress",
    "farm_server_poll", "farm_server_stats", "farm_server_free",
)
MLP_HIDDEN = 256
PHASES = ("normalize", "gemm", "pair", "topk", "rescore", "explain", "propose", "fallback", "select")

_STATUS = {FARM_ERR_INVALID_ARG: "invalid argument", FARM_ERR_OOM: "out of memory", FARM_ERR_HIP: "HIP error",
           FARM_ERR_UNSUPPORTED: "unsupported", FARM_ERR_BUSY: "busy"}


class FarmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class ServerConfig(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_int32), ("max_batch_q", ctypes.c_int32), ("max_batch_rel", ctypes.c_int32),
                ("k", ctypes.c_int32), ("dtype", ctypes.c_int32), ("method", ctypes.c_int32),
                ("hbm_budget", ctypes.c_size_t)]


class RrfChannel(ctypes.Structure):
    _fields_ = [("space", ctypes.c_int32), ("weight", ctypes.c_float), ("target", ctypes.c_void_p),
                ("anchor", ctypes.c_void_p)]


class ScoreOpts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int32), ("method", ctypes.c_int32), ("rescore_mult", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("certified", ctypes.c_void_p)]


def lib_path() -> str:
    return _PATH


def _declare(lib):
    P, i64, i32, u32, f32, sz = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32,
                                 ctypes.c_float, ctypes.c_size_t)
    pp = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "farm_build_memory": [i64, i32, P, P, P, P, P, f32, f32, u32, P, pp],
        "farm_set_entity_geometry": [P, P, P, P],
        "farm_add_embedding_space": [P, i32, P, P, P],
        "farm_rrf_similarity": [P, P, i32, i32, P, P, P, P, P, P],
        "farm_query_topk_rrf": [P, P, i32, i32, P, P, P, P, P, i32, P, P, P, P, P],
        "farm_free_memory": [P],
        "farm_memory_info": [P, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(sz)],
        "farm_workspace_create": [P, i32, i32, i32, pp],
        "farm_workspace_free": [P],
        "farm_workspace_bytes": [P, ctypes.POINTER(sz)],
        "farm_workspace_estimate": [P, i32, i32, i32, ctypes.POINTER(sz)],
        "farm_score_query": [P, P, i32, i32, P, P, P, P, P, P, P, P, P],
        "farm_similarity": [P, P, i32, i32, P, P, i32, P, P],
        "farm_topk": [P, P, P, i32, i32, P, P, P, P],
        "farm_query_topk": [P, P, i32, i32, P, P, P, P, P, ctypes.POINTER(ScoreOpts), i32, P, P, P, P, P],
        "farm_query_topk_static": [P, i32, i32, P, P, P, P, P, ctypes.POINTER(ScoreOpts), i32, P, P, P, P, P],
        "farm_workspace_status": [P, P],
        "farm_workspace_set_timing": [P, i32],
        "farm_workspace_timings": [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), i32],
        "farm_mlp_create": [i32, i32, ctypes.c_uint64, pp],
        "farm_mlp_free": [P],
        "farm_mlp_shape": [P, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "farm_mlp_get_weights": [P, P, P, P, P, P, P],
        "farm_mlp_get_grads": [P, P, P, P, P, P, P],
        "farm_mlp_set_weights": [P, P, P, P, P, P, P],
        "farm_mlp_get_batch": [P, i32, P, P, P, P, P, P, P, P],
        "farm_mlp_table_logits": [P, P, i64, i32, P, P],
        "farm_mlp_inputs": [P, P, i32, P, P, P, P],
        "farm_mlp_logits": [P, P, i32, P, P, P, P],
        "farm_mlp_step": [P, P, i32, P, P, P, P, ctypes.c_float, ctypes.c_float, i32, P, P],
        "farm_build_proposals": [P, P, i32, P],
        "farm_build_proposals_by_value": [P, i32, P],
        "farm_workspace_proposal_stats": [P, ctypes.POINTER(i64), i32, P],
        "farm_get_proposals": [P, ctypes.POINTER(i32), P, P, P, P],
        "farm_proposal_pass_form": [P, i32, ctypes.POINTER(i32)],
        "farm_server_create": [ctypes.POINTER(ServerConfig), pp],
        "farm_server_add_scene": [P, P, ctypes.POINTER(i32)],
        "farm_server_submit": [P, i32, i32, P, i32, i32, P, P, ctypes.POINTER(ctypes.c_uint64)],
        "farm_server_cancel": [P, ctypes.c_uint64],
        "farm_server_progress": [P, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "farm_server_poll": [P, i32, P, P, P, P, P, P, ctypes.POINTER(i32)],
        "farm_server_stats": [P, ctypes.POINTER(i64)],
        "farm_server_free": [P],
        "farm_last_error": [],
        "farm_version": [],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name in ("farm_last_error", "farm_version") else ctypes.c_int
    return lib


def load(path: str | None = None):
    path = path or _PATH
    if not os.path.exists(path):
        raise ImportError(f"libfarm.so not built at {path}; run `python paper_2606_15476_amd/build.py` "
                          "(the HIP library is required: there is no fallback)")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7).
    # Loading torch first makes libfarm bind to that one instance; loading
    # libfarm first would bring in a second HIP/HSA runtime, and the second one
    # to initialise in the process finds no device.
    import torch  # noqa: F401
    return _declare(ctypes.CDLL(path))


L = load()


def check(status: int):
    if status != FARM_OK:
        msg = L.farm_last_error()
        raise FarmError(status, msg.decode() if msg else "")
