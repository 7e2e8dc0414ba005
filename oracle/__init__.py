"""CPU FP64 oracle for FARM's query-time relational scoring.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package. It shares no code with
the GPU library (``paper_2606_15476_amd``) and never imports it.

The arithmetic lives in ``farm_oracle.c`` (plain loops, double precision); this
module builds it with gcc on first use and marshals numpy arrays. Every
function cites the passage it follows in the C source's header.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "farm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "libfarm_oracle.so")

MAX_REL = 8
NO_ID = 0xFFFFFFFF

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        # FARM_ORACLE_LIB names another build of farm_oracle.c (the mutation
        # test loads deliberately broken copies to show that the pins catch them)
        lib = ctypes.CDLL(os.environ.get("FARM_ORACLE_LIB") or build())
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        lib.farm_oracle_predicate.restype = ctypes.c_double
        lib.farm_oracle_predicate.argtypes = [ctypes.c_int, P, P, P, P, P]
        lib.farm_oracle_score.restype = ctypes.c_int
        lib.farm_oracle_score.argtypes = [i64, ctypes.c_int, P, P, P, P, P, P, i32, P, P, P, P, P, P, P, P, P]
        lib.farm_oracle_score_pairs.restype = ctypes.c_int
        lib.farm_oracle_score_pairs.argtypes = [i64, ctypes.c_int, P, P, P, P, P, P, i32, P, P, P, P, P,
                                                i64, P, P, P, P, P, P]
        lib.farm_oracle_topk.restype = ctypes.c_int
        lib.farm_oracle_topk.argtypes = [i64, P, P, i32, P]
        lib.farm_oracle_binding_value.restype = ctypes.c_double
        lib.farm_oracle_binding_value.argtypes = [i64, ctypes.c_int, P, P, P, P, P, P, i32, ctypes.c_int, P, i64,
                                                  i64]
        lib.farm_oracle_pair_features.restype = None
        lib.farm_oracle_pair_features.argtypes = [P, P, P, i64, i64, P]
        lib.farm_oracle_mlp.restype = ctypes.c_int
        lib.farm_oracle_mlp.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, i64, P, P, P, P,
                                        P, P, P, P, P, P, P]
        lib.farm_oracle_threads.restype = ctypes.c_int
        lib.farm_oracle_threads.argtypes = []
        lib.farm_oracle_set_threads.restype = None
        lib.farm_oracle_set_threads.argtypes = [ctypes.c_int]
        lib.farm_oracle_between.restype = ctypes.c_double
        lib.farm_oracle_between.argtypes = [P, P, P]
        lib.farm_oracle_between_binding_value.restype = ctypes.c_double
        lib.farm_oracle_between_binding_value.argtypes = [i64, ctypes.c_int, P, P, P, P, i64, i64, i64]
        lib.farm_oracle_set_between_tolerance.restype = None
        lib.farm_oracle_set_between_tolerance.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.farm_oracle_set_rank_tolerance.restype = None
        lib.farm_oracle_set_rank_tolerance.argtypes = [ctypes.c_int, ctypes.c_double]
        lib.farm_oracle_hellinger_near.restype = ctypes.c_double
        lib.farm_oracle_hellinger_near.argtypes = [P, P, P, P]
        lib.farm_oracle_view_predicate.restype = ctypes.c_double
        lib.farm_oracle_view_predicate.argtypes = [ctypes.c_int, P, P, P]
        lib.farm_oracle_set_similarities.restype = None
        lib.farm_oracle_set_similarities.argtypes = [i32, i32, i64, P, P]
        lib.farm_oracle_set_entity_geometry.restype = None
        lib.farm_oracle_set_entity_geometry.argtypes = [i64, P, P]
        lib.farm_oracle_topk_bounded.restype = ctypes.c_int
        lib.farm_oracle_topk_bounded.argtypes = [i64, ctypes.c_int, P, P, P, P, P, P, i32, P, P, P, P, P,
                                                 i32, P, P, P, P, P]
        _lib = lib
    return _lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def threads() -> int:
    """Threads the oracle's parallel loops use."""
    return int(_load().farm_oracle_threads())


class rank_tolerance:
    """Context manager: within it the rank predicates (Closest/Farthest) take
    the lowest (mode -1) or highest (mode +1) value over every rank that
    results when candidates whose squared distances to the anchor lie within a
    relative ``eps`` of the target's are ordered either way (a tie-aware check
    of an implementation that compares distances at lower precision).  Outside
    it the rank is exact (FP64 distances, ties by id)."""

    def __init__(self, mode: int, eps: float):
        self.mode, self.eps = int(mode), float(eps)

    def __enter__(self):
        _load().farm_oracle_set_rank_tolerance(self.mode, self.eps)
        return self

    def __exit__(self, *exc):
        _load().farm_oracle_set_rank_tolerance(0, 0.0)
        return False


class between_tolerance:
    """Context manager: within it Between's candidate sets keep only the
    anchors surely among the 64 of largest similarity (mode -1: more than
    ``eps`` above the 64th largest) or add every anchor within ``eps`` of it
    (mode +1), the lowest and highest terms an implementation whose
    similarities are within eps of the oracle's can return."""

    def __init__(self, mode: int, eps: float):
        self.mode, self.eps = int(mode), float(eps)

    def __enter__(self):
        _load().farm_oracle_set_between_tolerance(self.mode, self.eps)
        return self

    def __exit__(self, *exc):
        _load().farm_oracle_set_between_tolerance(0, 0.0)
        return False


BETWEEN_K = 64


def set_threads(n: int):
    """Threads of the oracle's parallel loops from now on."""
    _load().farm_oracle_set_threads(int(n))


def predicate(p: int, ci, cj, right, ei=(0.0, 0.0, 0.0), ej=(0.0, 0.0, 0.0)) -> float:
    """P_p(i, j) in FP64 for float32 centers, full extents (used by On only) and
    viewer right vector."""
    lib = _load()
    a, pa = _c(ci, np.float32)
    b, pb = _c(cj, np.float32)
    ea, pea = _c(ei, np.float32)
    eb, peb = _c(ej, np.float32)
    r, pr = _c(right, np.float32)
    return float(lib.farm_oracle_predicate(int(p), pa, pb, pea, peb, pr))


def between(ci, c1, c2) -> float:
    """Between(i; j1, j2) in FP64 for float32 centers of the target and the two anchors."""
    lib = _load()
    a, pa = _c(ci, np.float32)
    b, pb = _c(c1, np.float32)
    c, pc = _c(c2, np.float32)
    return float(lib.farm_oracle_between(pa, pb, pc))


def between_binding_value(scene, anchor1, anchor2, i: int, j1: int, j2: int) -> float:
    """sim(j1, q1) * sim(j2, q2) * Between(i; j1, j2) in FP64 for one binding of a Between invocation."""
    lib = _load()
    desc, pd = _c(scene.desc, np.float32)
    cen, pc = _c(scene.center, np.float32)
    a1, p1 = _c(anchor1, np.float32)
    a2, p2 = _c(anchor2, np.float32)
    return float(lib.farm_oracle_between_binding_value(int(desc.shape[0]), int(desc.shape[1]), pd, pc, p1, p2,
                                                       int(i), int(j1), int(j2)))


def hellinger_near(ci, cov_i, cj, cov_j) -> float:
    """Near over entity Gaussians, 1 - H(N(ci, cov_i), N(cj, cov_j)), FP64 from float32 centers and
    packed covariances (xx, xy, xz, yy, yz, zz)."""
    lib = _load()
    a, pa = _c(ci, np.float32)
    A, pA = _c(cov_i, np.float32)
    b, pb = _c(cj, np.float32)
    B, pB = _c(cov_j, np.float32)
    return float(lib.farm_oracle_hellinger_near(pa, pA, pb, pB))


def view_predicate(p: int, view_i, ci, cj) -> float:
    """A viewpoint-dependent predicate (15..18) of target center ci and anchor center cj in the
    target's stored view [camera center, right, down, forward axes], FP64 from float32 inputs."""
    lib = _load()
    v, pv = _c(view_i, np.float32)
    a, pa = _c(ci, np.float32)
    b, pb = _c(cj, np.float32)
    return float(lib.farm_oracle_view_predicate(int(p), pv, pa, pb))


class _geometry:
    """Context manager: the scene's entity Gaussians and stored views, when it has them, are what the
    oracle's scoring calls see inside it; cleared on exit."""

    def __init__(self, scene):
        self.cov = None if getattr(scene, "cov", None) is None else np.ascontiguousarray(scene.cov, np.float32)
        self.view = None if getattr(scene, "view", None) is None else np.ascontiguousarray(scene.view, np.float32)
        self.n = int(scene.desc.shape[0])

    def __enter__(self):
        ptr = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
        _load().farm_oracle_set_entity_geometry(self.n, ptr(self.cov), ptr(self.view))
        return self

    def __exit__(self, *exc):
        _load().farm_oracle_set_entity_geometry(-1, None, None)
        return False


def _scene_args(scene):
    desc, pd = _c(scene.desc, np.float32)
    cen, pc = _c(scene.center, np.float32)
    ext, pe = _c(scene.extent, np.float32)
    ids, pi = _c(scene.ids, np.uint32)
    if scene.cls is None:
        cls, pk = None, None
    else:
        cls, pk = _c(scene.cls, np.int32)
    vr, pv = _c(scene.view_right, np.float32)
    keep = (desc, cen, ext, ids, cls, vr)
    return keep, [int(desc.shape[0]), int(desc.shape[1]), pd, pc, pe, pi, pk, pv]


def _query_args(qb):
    tg, pt = _c(qb.target, np.float32)
    if qb.target_cls is None:
        tc, ptc = None, None
    else:
        tc, ptc = _c(qb.target_cls, np.int32)
    ro, pro = _c(qb.rel_off, np.int32)
    rp, prp = _c(qb.rel_pred, np.int32)
    ra, pra = _c(qb.rel_anchor.reshape(-1, qb.target.shape[1]) if qb.rel_anchor.size else
                 np.zeros((1, qb.target.shape[1]), np.float32), np.float32)
    keep = (tg, tc, ro, rp, ra)
    return keep, [int(tg.shape[0]), pt, ptc, pro, prp, pra]


class similarities:
    """Context manager: inside it the oracle's scoring calls take the unary scores from ``sem``
    [q, n] (target rows, class factor included) and ``asim`` [r_tot, n] (relation rows) instead of
    the clamped cosines of the query vectors (oracle/rrf.py's fused scores, for instance)."""

    def __init__(self, sem, asim):
        self.sem = np.ascontiguousarray(sem, np.float64)
        self.asim = np.ascontiguousarray(asim, np.float64).reshape(-1, self.sem.shape[1])

    def __enter__(self):
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a.size else None
        _load().farm_oracle_set_similarities(self.sem.shape[0], self.asim.shape[0], self.sem.shape[1],
                                             p(self.sem), p(self.asim))
        return self

    def __exit__(self, *exc):
        _load().farm_oracle_set_similarities(-1, -1, -1, None, None)
        return False


def score(scene, qb, terms: bool = False):
    """Full FP64 scores [q, n]; with ``terms`` also s_sem [q, n], t_r and b_r [r_tot, n]."""
    lib = _load()
    k1, sa = _scene_args(scene)
    k2, qa = _query_args(qb)
    n, q = sa[0], qa[0]
    r_tot = int(qb.rel_off[-1])
    out = np.zeros((q, n), np.float64)
    sem = np.zeros((q, n), np.float64) if terms else None
    t = np.zeros((r_tot, n), np.float64) if terms else None
    b = np.zeros((r_tot, n), np.uint32) if terms else None
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None and a.size else None
    with _geometry(scene):
        rc = lib.farm_oracle_score(*sa, *qa, ptr(out), ptr(sem), ptr(t), ptr(b))
    if rc:
        raise ValueError(f"oracle score failed ({rc})")
    del k1, k2
    return (out, sem, t, b) if terms else out


def score_pairs(scene, qb, qsel, osel):
    """FP64 scores of selected (query, object) pairs; returns (s, s_sem, t[m,8], b[m,8])."""
    lib = _load()
    k1, sa = _scene_args(scene)
    k2, qa = _query_args(qb)
    qs, pq = _c(qsel, np.int32)
    os_, po = _c(osel, np.int64)
    m = int(qs.shape[0])
    out = np.zeros(max(m, 1), np.float64)
    sem = np.zeros(max(m, 1), np.float64)
    t = np.zeros((max(m, 1), MAX_REL), np.float64)
    b = np.zeros((max(m, 1), MAX_REL), np.uint32)
    with _geometry(scene):
        rc = lib.farm_oracle_score_pairs(*sa, *qa, m, pq, po, out.ctypes.data_as(ctypes.c_void_p),
                                         sem.ctypes.data_as(ctypes.c_void_p), t.ctypes.data_as(ctypes.c_void_p),
                                         b.ctypes.data_as(ctypes.c_void_p))
    if rc:
        raise ValueError(f"oracle score_pairs failed ({rc})")
    del k1, k2
    return out[:m], sem[:m], t[:m], b[:m]


def topk(scores_row, ids, k: int):
    """Indices of the first min(k, n) objects by (score desc, id asc); -1 padding."""
    lib = _load()
    s, ps = _c(scores_row, np.float64)
    i, pi = _c(ids, np.uint32)
    out = np.zeros(k, np.int64)
    rc = lib.farm_oracle_topk(int(s.shape[0]), ps, pi, int(k), out.ctypes.data_as(ctypes.c_void_p))
    if rc:
        raise ValueError(f"oracle topk failed ({rc})")
    return out


def topk_bounded(scene, qb, k: int):
    """Exact TopK via the soft-blend bound; returns (idx[q,k], score[q,k], t[q,k,8], b[q,k,8], n_scored[q])."""
    lib = _load()
    k1, sa = _scene_args(scene)
    k2, qa = _query_args(qb)
    q = qa[0]
    idx = np.zeros((q, k), np.int64)
    sc = np.zeros((q, k), np.float64)
    t = np.zeros((q, k, MAX_REL), np.float64)
    b = np.zeros((q, k, MAX_REL), np.uint32)
    ns = np.zeros(q, np.int64)
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    with _geometry(scene):
        rc = lib.farm_oracle_topk_bounded(*sa, *qa, int(k), p(idx), p(sc), p(t), p(b), p(ns))
    if rc:
        raise ValueError(f"oracle topk_bounded failed ({rc})")
    del k1, k2
    return idx, sc, t, b, ns


def binding_value(scene, pred: int, anchor_vec, i: int, j: int, target_cls: int = -1) -> float:
    """sim(j, q_r) * P_pred(i, j) in FP64 for one candidate binding (target_cls:
    the query's parsed class, which fixes the candidate set of Closest/Farthest)."""
    lib = _load()
    desc, pd = _c(scene.desc, np.float32)
    cen, pc = _c(scene.center, np.float32)
    ext, pe = _c(scene.extent, np.float32)
    ids, pi = _c(scene.ids, np.uint32)
    if scene.cls is None:
        cls, pk = None, None
    else:
        cls, pk = _c(scene.cls, np.int32)
    vr, pv = _c(scene.view_right, np.float32)
    av, pa = _c(anchor_vec, np.float32)
    with _geometry(scene):
        return float(lib.farm_oracle_binding_value(int(desc.shape[0]), int(desc.shape[1]), pd, pc, pe, pi, pk, pv,
                                                   int(target_cls), int(pred), pa, int(i), int(j)))


NUM_PRED = 19  # predicate ids 0..18 (On = 8, Closest = 9, Farthest = 10, Inside = 11, Between = 12 and its
#               second anchor 13, Hellinger Near = 14, the stored-view LeftOf, RightOf, InFrontOf, Behind = 15..18)
NPRED = 9      # proposal-network outputs, one per predicate
NGEO = 12


def pair_features(scene, o: int, a: int):
    """The 12 relative-geometry features g(o, a) of the proposal network, FP64."""
    lib = _load()
    c, pc = _c(scene.center, np.float32)
    e, pe = _c(scene.extent, np.float32)
    r, pr = _c(scene.view_right, np.float32)
    g = np.zeros(NGEO, np.float64)
    lib.farm_oracle_pair_features(pc, pe, pr, int(o), int(a), g.ctypes.data_as(ctypes.c_void_p))
    return g


def mlp(weights: dict, X, pred, label, grads: bool = True):
    """Loss (mean BCE-with-logits on the labelled predicate), logits [n,9] and,
    with ``grads``, the FP64 gradients {name: array} of the proposal network.
    weights: W1 [h,in], b1 [h], W2 [h,h], b2 [h], W3 [9,h], b3 [9]."""
    lib = _load()
    W = {k: np.ascontiguousarray(v, np.float64) for k, v in weights.items()}
    h, inp = W["W1"].shape
    want = {"W1": (h, inp), "b1": (h,), "W2": (h, h), "b2": (h,), "W3": (NPRED, h), "b3": (NPRED,)}
    for k, shape in want.items():
        if W[k].shape != shape:
            raise ValueError(f"oracle mlp: {k} has shape {W[k].shape}, expected {shape}")
    Xa, px = _c(X, np.float64)
    pa, pp = _c(pred, np.int32)
    la, pl = _c(label, np.float64)
    n = int(Xa.shape[0])
    loss = ctypes.c_double()
    logits = np.zeros((n, NPRED), np.float64)
    g = {k: np.zeros_like(v) for k, v in W.items()} if grads else None
    ptr = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    rc = lib.farm_oracle_mlp(inp, h, ptr(W["W1"]), ptr(W["b1"]), ptr(W["W2"]), ptr(W["b2"]), ptr(W["W3"]),
                             ptr(W["b3"]), n, px, pp, pl, ctypes.byref(loss),
                             *(ptr(g[k]) if grads else None for k in ("W1", "b1", "W2", "b2", "W3", "b3")),
                             ptr(logits))
    if rc:
        raise ValueError(f"oracle mlp failed ({rc})")
    return float(loss.value), logits, g
