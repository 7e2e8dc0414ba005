"""MI355X-native FARM query-time relational retrieval.

Thin Python binding over libfarm.so (the C ABI declared in include/farm.h).
Every step of the scoring path runs in the library's HIP kernels; this module
only marshals arguments: torch CUDA tensors become device pointers, numpy
arrays become host pointers, torch streams become hipStream_t handles.
There is no CPU fallback: if the library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _lib
from ._lib import (FARM_BUILD_BF16, FARM_BUILD_FP8, FARM_MAX_K, FARM_MAX_REL, FARM_NO_ID, F32, BF16, FP8_E4M3,
                   EXHAUSTIVE, BOUNDED, PROPOSAL, OPT_GLOBAL_PROPOSAL_PASS,
                   NEAR, ABOVE, BELOW, LEFT_OF, RIGHT_OF, NEXT_TO, IN_FRONT_OF, BEHIND, ON, CLOSEST,
                   FARTHEST, INSIDE, BETWEEN, AND, NEAR_HELLINGER, LEFT_OF_VIEW, RIGHT_OF_VIEW,
                   IN_FRONT_OF_VIEW, BEHIND_VIEW, NUM_PRED, NUM_PROP_PRED, FarmError, lib_path)

__all__ = [
    "Memory", "Workspace", "ProposalNet", "Server", "build_proposals", "build_proposals_by_value", "get_proposals", "score_query", "similarity", "topk", "query_topk", "rrf_similarity", "query_topk_rrf", "query_topk_static", "workspace_estimate", "FarmError",
    "FARM_BUILD_BF16", "FARM_BUILD_FP8", "FARM_MAX_K", "FARM_MAX_REL", "FARM_NO_ID", "F32", "BF16",
    "FP8_E4M3", "EXHAUSTIVE", "BOUNDED", "PROPOSAL", "OPT_GLOBAL_PROPOSAL_PASS", "NEAR", "ABOVE", "BELOW", "LEFT_OF", "RIGHT_OF", "NEXT_TO", "IN_FRONT_OF", "BEHIND", "ON", "CLOSEST", "FARTHEST", "INSIDE", "BETWEEN", "AND", "NEAR_HELLINGER", "LEFT_OF_VIEW", "RIGHT_OF_VIEW", "IN_FRONT_OF_VIEW", "BEHIND_VIEW", "NUM_PRED",
    "NUM_PROP_PRED", "lib_path",
]


def _ptr(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device (cuda) tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _host_i32(a):
    if a is None:
        return None, None
    arr = np.ascontiguousarray(np.asarray(a), dtype=np.int32)
    return arr, arr.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    handle = getattr(stream, "cuda_stream", stream)
    return ctypes.c_void_p(int(handle)) if handle else None


class Memory:
    """Device-resident scene (farm_build_memory)."""

    def __init__(self, desc, center, extent, ids, cls, view_right, flags: int = 0, stream=None):
        import torch
        n, d = int(desc.shape[0]), int(desc.shape[1])
        for name, t, dt in (("desc", desc, torch.float32), ("center", center, torch.float32),
                            ("extent", extent, torch.float32)):
            if t.dtype != dt:
                raise ValueError(f"{name} must be {dt}")
        if ids.dtype not in (torch.int32, getattr(torch, "uint32", torch.int32)):
            raise ValueError("ids must be a 32-bit integer tensor (bit pattern of uint32)")
        if cls is not None and cls.dtype != torch.int32:
            raise ValueError("cls must be int32")
        h = ctypes.c_void_p()
        _lib.check(_lib.L.farm_build_memory(n, d, _ptr(desc), _ptr(center), _ptr(extent), _ptr(ids), _ptr(cls),
                                            float(view_right[0]), float(view_right[1]), int(flags),
                                            _stream(stream), ctypes.byref(h)))
        self._h = h
        self.n, self.d, self.flags = n, d, int(flags)
        self.device = desc.device

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("memory was freed")
        return self._h

    def add_embedding_space(self, desc, stream=None) -> int:
        """farm_add_embedding_space: another per-entity embedding table desc [n, d] (FP32 device
        tensor); returns its space index (1, 2, ...)."""
        import torch
        if desc.dtype != torch.float32 or desc.dim() != 2 or int(desc.shape[0]) != self.n or not desc.is_contiguous():
            raise ValueError(f"desc must be a contiguous float32 [{self.n}, d] tensor")
        sp = ctypes.c_int32()
        _lib.check(_lib.L.farm_add_embedding_space(self.handle, int(desc.shape[1]), _ptr(desc), _stream(stream),
                                                   ctypes.byref(sp)))
        return int(sp.value)

    def set_entity_geometry(self, cov=None, view=None, stream=None):
        """farm_set_entity_geometry: entity Gaussians cov [n, 6] (packed xx, xy, xz, yy, yz, zz) and
        stored views view [n, 12] (camera center, right, down, forward axes), FP32 device tensors;
        either may be None (kept as it is)."""
        import torch
        for name, t, w in (("cov", cov, 6), ("view", view, 12)):
            if t is not None and (t.dtype != torch.float32 or tuple(t.shape) != (self.n, w) or not t.is_contiguous()):
                raise ValueError(f"{name} must be a contiguous float32 [{self.n}, {w}] tensor")
        _lib.check(_lib.L.farm_set_entity_geometry(self.handle, _ptr(cov), _ptr(view), _stream(stream)))

    @property
    def bytes(self) -> int:
        b = ctypes.c_size_t()
        _lib.check(_lib.L.farm_memory_info(self.handle, None, None, ctypes.byref(b)))
        return int(b.value)

    def proposal_pass_in_lds(self, dtype: int = F32) -> bool:
        """Whether FARM_METHOD_PROPOSAL stages similarity rows in LDS on this memory."""
        v = ctypes.c_int32()
        _lib.check(_lib.L.farm_proposal_pass_form(self.handle, int(dtype), ctypes.byref(v)))
        return bool(v.value)

    def close(self):
        """Free the device memory.  Raises FarmError (FARM_ERR_BUSY) while
        workspaces or servers still use it; the handle then stays valid."""
        if getattr(self, "_h", None) is not None:
            _lib.check(_lib.L.farm_free_memory(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Workspace:
    """Per-stream scratch for scoring calls (farm_workspace_create)."""

    def __init__(self, mem: Memory, max_q: int, max_rel: int, max_k: int = 64):
        h = ctypes.c_void_p()
        _lib.check(_lib.L.farm_workspace_create(mem.handle, int(max_q), int(max_rel), int(max_k), ctypes.byref(h)))
        self._h = h
        self.mem = mem
        self.max_q, self.max_rel, self.max_k = int(max_q), int(max_rel), int(max_k)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("workspace was freed")
        return self._h

    @property
    def bytes(self) -> int:
        b = ctypes.c_size_t()
        _lib.check(_lib.L.farm_workspace_bytes(self.handle, ctypes.byref(b)))
        return int(b.value)

    def set_timing(self, enable: bool = True):
        """Enable the native per-phase HIP-event timer of this workspace."""
        _lib.check(_lib.L.farm_workspace_set_timing(self.handle, 1 if enable else 0))

    def timings(self, reset: bool = False) -> dict:
        """{phase: (total_ms, launches)} accumulated by the phase timer."""
        ms = (ctypes.c_double * len(_lib.PHASES))()
        cnt = (ctypes.c_int64 * len(_lib.PHASES))()
        _lib.check(_lib.L.farm_workspace_timings(self.handle, ms, cnt, 1 if reset else 0))
        return {p: (float(ms[i]), int(cnt[i])) for i, p in enumerate(_lib.PHASES)}

    def status(self, stream=None):
        _lib.check(_lib.L.farm_workspace_status(self.handle, _stream(stream)))

    def proposal_stats(self, reset: bool = False, stream=None) -> tuple:
        """(terms evaluated, terms that fell back to the full anchor scan, FP32 dot products in the
        proposal pass, FP32 dot products in the fallback scans) under method PROPOSAL."""
        out = (ctypes.c_int64 * 4)()
        _lib.check(_lib.L.farm_workspace_proposal_stats(self.handle, out, 1 if reset else 0, _stream(stream)))
        return tuple(int(v) for v in out)

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.L.farm_workspace_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_estimate(mem: Memory, max_q: int, max_rel: int, max_k: int = 64) -> int:
    b = ctypes.c_size_t()
    _lib.check(_lib.L.farm_workspace_estimate(mem.handle, int(max_q), int(max_rel), int(max_k), ctypes.byref(b)))
    return int(b.value)


def score_query(mem: Memory, ws: Workspace, target, target_cls, rel_off, rel_pred, rel_anchor, scores,
                rel_terms=None, rel_anchor_id=None, stream=None):
    """farm_score_query: full score rows (and optional t_r, b_r) into caller tensors."""
    tc, ptc = _host_i32(target_cls)
    ro, pro = _host_i32(rel_off)
    rp, prp = _host_i32(rel_pred)
    q, d = int(target.shape[0]), int(target.shape[1])
    _lib.check(_lib.L.farm_score_query(mem.handle, ws.handle, q, d, _ptr(target), ptc, pro, prp,
                                       _ptr(rel_anchor) if rel_anchor is not None and rel_anchor.numel() else None,
                                       _ptr(scores), _ptr(rel_terms), _ptr(rel_anchor_id), _stream(stream)))
    del tc, ro, rp


def similarity(mem: Memory, ws: Workspace, target, target_cls, out, dtype: int = F32, stream=None):
    """farm_similarity: the similarity GEMM's s_sem rows in `dtype` into out [q][n]."""
    tc, ptc = _host_i32(target_cls)
    q, d = int(target.shape[0]), int(target.shape[1])
    _lib.check(_lib.L.farm_similarity(mem.handle, ws.handle, q, d, _ptr(target), ptc, int(dtype), _ptr(out),
                                      _stream(stream)))
    del tc


def topk(mem: Memory, ws: Workspace, scores, k: int, out_id, out_score, out_index=None, stream=None):
    """farm_topk over precomputed score rows."""
    q = int(scores.shape[0])
    _lib.check(_lib.L.farm_topk(mem.handle, ws.handle, _ptr(scores), q, int(k), _ptr(out_id), _ptr(out_score),
                                _ptr(out_index), _stream(stream)))


def query_topk(mem: Memory, ws: Workspace, target, target_cls, rel_off, rel_pred, rel_anchor, k: int, out_id,
               out_score, out_terms=None, out_anchor_id=None, dtype: int = F32, rescore_mult: int = 4,
               certified=None, method: int = EXHAUSTIVE, flags: int = 0, stream=None):
    """farm_query_topk: fused scoring + TopK + ScoredCandidate breakdown."""
    tc, ptc = _host_i32(target_cls)
    ro, pro = _host_i32(rel_off)
    rp, prp = _host_i32(rel_pred)
    q, d = int(target.shape[0]), int(target.shape[1])
    cp = _ptr(certified)
    opts = _lib.ScoreOpts(int(dtype), int(method), int(rescore_mult), int(flags), cp.value if cp is not None else None)
    _lib.check(_lib.L.farm_query_topk(mem.handle, ws.handle, q, d, _ptr(target), ptc, pro, prp,
                                      _ptr(rel_anchor) if rel_anchor is not None and rel_anchor.numel() else None,
                                      ctypes.byref(opts), int(k), _ptr(out_id), _ptr(out_score), _ptr(out_terms),
                                      _ptr(out_anchor_id), _stream(stream)))
    del tc, ro, rp


def _channels(channels):
    """[(space, weight, target [q, d_s] tensor, anchor [R, d_s] tensor or None)] -> ctypes array (+ q)."""
    arr = (_lib.RrfChannel * len(channels))()
    q = None
    for i, (sp, w, tgt, anc) in enumerate(channels):
        q = int(tgt.shape[0]) if q is None else q
        if int(tgt.shape[0]) != q:
            raise ValueError("every channel needs the same number of target rows")
        arr[i] = _lib.RrfChannel(int(sp), float(w), _ptr(tgt),
                                 _ptr(anc) if anc is not None and anc.numel() else None)
    return arr, q


def rrf_similarity(mem: Memory, ws: Workspace, channels, target_cls, rel_off, rel_pred, out, stream=None):
    """farm_rrf_similarity: the fused unary rows [q + R, n] into out."""
    arr, q = _channels(channels)
    tc, ptc = _host_i32(target_cls)
    ro, pro = _host_i32(rel_off)
    rp, prp = _host_i32(rel_pred)
    _lib.check(_lib.L.farm_rrf_similarity(mem.handle, ws.handle, q, len(channels), arr, ptc, pro, prp, _ptr(out),
                                          _stream(stream)))
    del tc, ro, rp


def query_topk_rrf(mem: Memory, ws: Workspace, channels, target_cls, rel_off, rel_pred, k: int, out_id, out_score,
                   out_terms=None, out_anchor_id=None, certified=None, method: int = EXHAUSTIVE, dtype: int = F32,
                   stream=None):
    """farm_query_topk_rrf: fused scoring + TopK with multi-channel reciprocal-rank fusion unary scores."""
    arr, q = _channels(channels)
    tc, ptc = _host_i32(target_cls)
    ro, pro = _host_i32(rel_off)
    rp, prp = _host_i32(rel_pred)
    cp = _ptr(certified)
    opts = _lib.ScoreOpts(int(dtype), int(method), 4, 0, cp.value if cp is not None else None)
    _lib.check(_lib.L.farm_query_topk_rrf(mem.handle, ws.handle, q, len(channels), arr, ptc, pro, prp,
                                          ctypes.byref(opts), int(k), _ptr(out_id), _ptr(out_score), _ptr(out_terms),
                                          _ptr(out_anchor_id), _stream(stream)))
    del tc, ro, rp


def query_topk_static(mem: Memory, target, target_cls, rel_off, rel_pred, rel_anchor, k: int, out_id, out_score,
                      out_terms=None, out_anchor_id=None, dtype: int = F32, rescore_mult: int = 4, certified=None,
                      method: int = EXHAUSTIVE, flags: int = 0, stream=None):
    """farm_query_topk_static: query_topk without a workspace or any allocation (the library's static scratch)."""
    tc, ptc = _host_i32(target_cls)
    ro, pro = _host_i32(rel_off)
    rp, prp = _host_i32(rel_pred)
    q, d = int(target.shape[0]), int(target.shape[1])
    cp = _ptr(certified)
    opts = _lib.ScoreOpts(int(dtype), int(method), int(rescore_mult), int(flags), cp.value if cp is not None else None)
    _lib.check(_lib.L.farm_query_topk_static(mem.handle, q, d, _ptr(target), ptc, pro, prp,
                                             _ptr(rel_anchor) if rel_anchor is not None and rel_anchor.numel() else None,
                                             ctypes.byref(opts), int(k), _ptr(out_id), _ptr(out_score),
                                             _ptr(out_terms), _ptr(out_anchor_id), _stream(stream)))
    del tc, ro, rp


def build_proposals(mem: Memory, net: "ProposalNet", m: int = 256, stream=None):
    """farm_build_proposals: per-(object, predicate) anchor lists of length m from the network."""
    _lib.check(_lib.L.farm_build_proposals(mem.handle, net.handle, int(m), _stream(stream)))


def build_proposals_by_value(mem: Memory, m: int = 256, stream=None):
    """farm_build_proposals_by_value: lists of the m anchors of largest exact predicate value (no network)."""
    _lib.check(_lib.L.farm_build_proposals_by_value(mem.handle, int(m), _stream(stream)))


def get_proposals(mem: Memory, stream=None):
    """(M, idx [P,n,M] int32, val [P,n,M] float32, out [P,n] float32) device tensors (P = NUM_PROP_PRED), or
    (0, None, None, None)."""
    import torch
    m = ctypes.c_int32()
    _lib.check(_lib.L.farm_get_proposals(mem.handle, ctypes.byref(m), None, None, None, _stream(stream)))
    if m.value == 0:
        return 0, None, None, None
    n = mem.n
    idx = torch.empty((NUM_PROP_PRED, n, m.value), dtype=torch.int32, device=mem.device)
    val = torch.empty((NUM_PROP_PRED, n, m.value), dtype=torch.float32, device=mem.device)
    out = torch.empty((NUM_PROP_PRED, n), dtype=torch.float32, device=mem.device)
    _lib.check(_lib.L.farm_get_proposals(mem.handle, ctypes.byref(m), _ptr(idx), _ptr(val), _ptr(out),
                                         _stream(stream)))
    return m.value, idx, val, out


class ProposalNet:
    """The anchor proposal network (farm_mlp_*): BF16 GEMMs, FP32 masters, AdamW."""

    PARAMS = ("W1", "b1", "W2", "b2", "W3", "b3")

    def __init__(self, d: int, max_batch: int = 8192, seed: int = 0):
        h = ctypes.c_void_p()
        _lib.check(_lib.L.farm_mlp_create(int(d), int(max_batch), int(seed), ctypes.byref(h)))
        self._h = h
        self.d, self.max_batch = int(d), int(max_batch)
        ind, hid = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.L.farm_mlp_shape(h, ctypes.byref(ind), ctypes.byref(hid)))
        self.in_dim, self.hidden = int(ind.value), int(hid.value)

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("network was freed")
        return self._h

    def _shapes(self):
        h, i = self.hidden, self.in_dim
        return {"W1": (h, i), "b1": (h,), "W2": (h, h), "b2": (h,), "W3": (NUM_PROP_PRED, h), "b3": (NUM_PROP_PRED,)}

    def _io(self, fn, arrays):
        ptrs = [arrays[k].ctypes.data_as(ctypes.c_void_p) for k in self.PARAMS]
        _lib.check(fn(self.handle, *ptrs))
        return arrays

    def weights(self) -> dict:
        return self._io(_lib.L.farm_mlp_get_weights, {k: np.zeros(v, np.float32) for k, v in self._shapes().items()})

    def grads(self) -> dict:
        return self._io(_lib.L.farm_mlp_get_grads, {k: np.zeros(v, np.float32) for k, v in self._shapes().items()})

    def set_weights(self, w: dict):
        arrays = {k: np.ascontiguousarray(w[k], np.float32).reshape(v) for k, v in self._shapes().items()}
        self._io(_lib.L.farm_mlp_set_weights, arrays)

    def batch(self, nb: int) -> dict:
        """Host copies of the last step's batch tensors (farm_mlp_get_batch): Z1, Z2, dA1 FP32 [nb, h],
        A1, A2, dZ2, dZ1 as BF16 bit patterns (uint16) [nb, h], Y FP32 [nb, NUM_PROP_PRED]."""
        h = self.hidden
        out = {"Z1": np.zeros((nb, h), np.float32), "A1": np.zeros((nb, h), np.uint16),
               "Z2": np.zeros((nb, h), np.float32), "A2": np.zeros((nb, h), np.uint16),
               "Y": np.zeros((nb, NUM_PROP_PRED), np.float32), "dZ2": np.zeros((nb, h), np.uint16),
               "dA1": np.zeros((nb, h), np.float32), "dZ1": np.zeros((nb, h), np.uint16)}
        ptrs = [out[k].ctypes.data_as(ctypes.c_void_p) for k in ("Z1", "A1", "Z2", "A2", "Y", "dZ2", "dA1", "dZ1")]
        _lib.check(_lib.L.farm_mlp_get_batch(self.handle, int(nb), *ptrs))
        return out

    def table_logits(self, mem: "Memory", t0: int, tc: int, out, stream=None):
        """farm_mlp_table_logits: the table build's logits [NUM_PROP_PRED, tc, n] of targets t0..t0+tc-1."""
        _lib.check(_lib.L.farm_mlp_table_logits(self.handle, mem.handle, int(t0), int(tc), _ptr(out), _stream(stream)))

    def inputs(self, mem: "Memory", o_idx, a_idx, out, stream=None):
        _lib.check(_lib.L.farm_mlp_inputs(self.handle, mem.handle, int(o_idx.shape[0]), _ptr(o_idx), _ptr(a_idx),
                                          _ptr(out), _stream(stream)))

    def logits(self, mem: "Memory", o_idx, a_idx, out, stream=None):
        _lib.check(_lib.L.farm_mlp_logits(self.handle, mem.handle, int(o_idx.shape[0]), _ptr(o_idx), _ptr(a_idx),
                                          _ptr(out), _stream(stream)))

    def step(self, mem: "Memory", o_idx, a_idx, pred, label, lr: float = 1e-3, weight_decay: float = 0.0,
             update: bool = True, loss_out=None, stream=None):
        _lib.check(_lib.L.farm_mlp_step(self.handle, mem.handle, int(o_idx.shape[0]), _ptr(o_idx), _ptr(a_idx),
                                        _ptr(pred), _ptr(label), float(lr), float(weight_decay), 1 if update else 0,
                                        _ptr(loss_out), _stream(stream)))

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.L.farm_mlp_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Request loop over resident scenes (farm_server_*): continuous batching,
    HBM-budget admission, one stream per slot.  Driven by progress()."""

    def __init__(self, slots: int = 4, max_batch_q: int = 64, max_batch_rel: int = 256, k: int = 10,
                 dtype: int = F32, method: int = EXHAUSTIVE, hbm_budget: int = 8 << 30):
        cfg = _lib.ServerConfig(int(slots), int(max_batch_q), int(max_batch_rel), int(k), int(dtype), int(method),
                                int(hbm_budget))
        h = ctypes.c_void_p()
        _lib.check(_lib.L.farm_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.k = int(k)
        self.scenes = []

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("server was freed")
        return self._h

    def add_scene(self, mem: Memory) -> int:
        idx = ctypes.c_int32()
        _lib.check(_lib.L.farm_server_add_scene(self.handle, mem.handle, ctypes.byref(idx)))
        self.scenes.append(mem)
        return int(idx.value)

    def submit(self, scene: int, target, target_cls: int, preds, anchors) -> int:
        t = np.ascontiguousarray(target, dtype=np.float32).reshape(-1)
        p = np.ascontiguousarray(np.asarray(preds, dtype=np.int32).reshape(-1))
        a = np.ascontiguousarray(anchors, dtype=np.float32).reshape(-1)
        rid = ctypes.c_uint64()
        _lib.check(_lib.L.farm_server_submit(self.handle, int(scene), int(t.size), t.ctypes.data_as(ctypes.c_void_p),
                                             int(target_cls), int(p.size), p.ctypes.data_as(ctypes.c_void_p),
                                             a.ctypes.data_as(ctypes.c_void_p), ctypes.byref(rid)))
        return int(rid.value)

    def cancel(self, request_id: int):
        _lib.check(_lib.L.farm_server_cancel(self.handle, ctypes.c_uint64(int(request_id))))

    def progress(self) -> tuple:
        """(busy slots, pending requests) after reaping and admitting."""
        b, p = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.L.farm_server_progress(self.handle, ctypes.byref(b), ctypes.byref(p)))
        return int(b.value), int(p.value)

    def poll(self, max_results: int = 1024) -> list:
        """Completed requests: [(id, status, certified, latency_ns, ids[k] uint32, scores[k])]."""
        m, k = int(max_results), self.k
        ids = np.zeros(m, np.uint64)
        st = np.zeros(m, np.int32)
        ce = np.zeros(m, np.int32)
        lat = np.zeros(m, np.int64)
        tid = np.zeros((m, k), np.uint32)
        tsc = np.zeros((m, k), np.float32)
        n = ctypes.c_int32()
        vp = lambda x: x.ctypes.data_as(ctypes.c_void_p)
        _lib.check(_lib.L.farm_server_poll(self.handle, m, vp(ids), vp(st), vp(ce), vp(lat), vp(tid), vp(tsc),
                                           ctypes.byref(n)))
        return [(int(ids[i]), int(st[i]), int(ce[i]), int(lat[i]), tid[i].copy(), tsc[i].copy())
                for i in range(n.value)]

    def stats(self) -> dict:
        out = (ctypes.c_int64 * 5)()
        _lib.check(_lib.L.farm_server_stats(self.handle, out))
        return {"batches": out[0], "deferrals": out[1], "evictions": out[2], "bytes_held": out[3],
                "workspaces_held": out[4]}

    def close(self):
        if getattr(self, "_h", None) is not None:
            _lib.L.farm_server_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
