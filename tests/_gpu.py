"""Helpers that move synthetic scenes/queries to the GPU and call the C ABI.

Only marshalling: every computation runs in libfarm.so."""
import numpy as np


def device():
    import torch
    return torch.device("cuda:0")


def to_dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(device())


def build_memory(scene, flags=0):
    import torch
    import paper_2606_15476_amd as farm
    ids = to_dev(scene.ids.view(np.int32))
    cls = to_dev(scene.cls) if scene.cls is not None else None
    mem = farm.Memory(to_dev(scene.desc), to_dev(scene.center), to_dev(scene.extent), ids, cls,
                      scene.view_right, flags=flags)
    cov, view = getattr(scene, "cov", None), getattr(scene, "view", None)
    if cov is not None or view is not None:
        mem.set_entity_geometry(None if cov is None else to_dev(cov), None if view is None else to_dev(view))
    return mem


def query_tensors(qb):
    import torch
    d = qb.target.shape[1]
    target = to_dev(qb.target)
    anchors = to_dev(qb.rel_anchor.reshape(-1, d)) if qb.r_tot else torch.zeros((0, d), dtype=torch.float32,
                                                                                    device=device())
    return target, anchors


def score_full(mem, ws, qb, terms=True):
    """(scores [q,n], rel_terms [R,n], anchor_id [R,n]) as numpy."""
    import torch
    import paper_2606_15476_amd as farm
    target, anchors = query_tensors(qb)
    q, n, R = qb.q, mem.n, qb.r_tot
    scores = torch.empty((q, n), dtype=torch.float32, device=device())
    rt = torch.empty((max(R, 1), n), dtype=torch.float32, device=device()) if terms else None
    rb = torch.empty((max(R, 1), n), dtype=torch.int32, device=device()) if terms else None
    farm.score_query(mem, ws, target, qb.target_cls, qb.rel_off, qb.rel_pred, anchors, scores,
                     rt if terms and R else None, rb if terms and R else None)
    torch.cuda.synchronize()
    s = scores.cpu().numpy()
    if not terms:
        return s
    t = rt.cpu().numpy()[:R] if R else np.zeros((0, n), np.float32)
    b = rb.cpu().numpy().view(np.uint32)[:R] if R else np.zeros((0, n), np.uint32)
    return s, t, b


def query_topk(mem, ws, qb, k, dtype=0, rescore_mult=4, with_cert=False, method=0, flags=0):
    """(ids [q,k] uint32, scores [q,k], terms [q,k,8], anchor ids [q,k,8] uint32[, certified [q]]) as numpy."""
    import torch
    import paper_2606_15476_amd as farm
    target, anchors = query_tensors(qb)
    q = qb.q
    oid = torch.empty((q, k), dtype=torch.int32, device=device())
    osc = torch.empty((q, k), dtype=torch.float32, device=device())
    ot = torch.empty((q, k, 8), dtype=torch.float32, device=device())
    ob = torch.empty((q, k, 8), dtype=torch.int32, device=device())
    cert = torch.full((q,), -1, dtype=torch.int32, device=device())
    farm.query_topk(mem, ws, target, qb.target_cls, qb.rel_off, qb.rel_pred, anchors, k, oid, osc, ot, ob,
                    dtype=dtype, rescore_mult=rescore_mult, certified=cert, method=method, flags=flags)
    torch.cuda.synchronize()
    out = (oid.cpu().numpy().view(np.uint32), osc.cpu().numpy(), ot.cpu().numpy(), ob.cpu().numpy().view(np.uint32))
    return out + (cert.cpu().numpy(),) if with_cert else out
