"""Training data and training loop of the anchor proposal network.

The network (farm_mlp_*, kernels in csrc/mlp.hip) scores (target o, anchor a)
pairs with one logit per predicate; farm_build_proposals keeps the M best
anchors per (o, predicate).  It is trained on what the method itself outputs:
the exhaustive relational pass (farm_score_query) returns, for every relation
r of a training query and every object o, the binding b_r(o) -- the anchor that
attains the relation term, the greedy star binding of the paper's relational
retrieval (Appendix "Robust Relational Retrieval Formulation").  A pair
(o, b_r(o)) is a positive example for predicate p_r; anchors drawn uniformly
from the scene are negatives.  The network sees no query features, so it
learns which anchors tend to bind for each target and predicate: mostly
geometry (near anchors for Near, anchors under the target for Above, ...).

All arithmetic (scoring, forward, backward, AdamW) runs in libfarm's kernels;
this module draws the example indices on the host and marshals them.
"""
from __future__ import annotations

import numpy as np

from . import FARM_NO_ID, NUM_PROP_PRED, Memory, ProposalNet, Workspace, score_query


def exhaustive_bindings(mem: Memory, ws: Workspace, target, target_cls, rel_off, rel_pred, anchors, stream=None):
    """b_r(o) for every relation row r and object o, as object ids ([R, n] uint32 numpy)."""
    import torch
    q, n = int(target.shape[0]), mem.n
    R = int(np.asarray(rel_off)[-1])
    scores = torch.empty((q, n), dtype=torch.float32, device=target.device)
    terms = torch.empty((max(R, 1), n), dtype=torch.float32, device=target.device)
    bind = torch.empty((max(R, 1), n), dtype=torch.int32, device=target.device)
    score_query(mem, ws, target, target_cls, rel_off, rel_pred, anchors, scores, terms if R else None,
                bind if R else None, stream=stream)
    torch.cuda.synchronize()
    return bind.cpu().numpy().view(np.uint32)[:R]


def sample_pairs(bind_ids: np.ndarray, ids: np.ndarray, rel_pred: np.ndarray, rng: np.random.Generator,
                 per_relation: int = 64, negatives: int = 3):
    """Labelled (o, a, predicate, label) examples from the bindings of each relation row.

    For each relation row, `per_relation` targets o drawn uniformly give one
    positive (o, b_r(o)) each and `negatives` pairs (o, a) with a drawn
    uniformly (a != o; labelled 1 if it happens to be b_r(o)).  Rows of
    predicates the network has no output for (ids >= NUM_PROP_PRED) are
    skipped: their terms are scanned over all anchors."""
    R, n = bind_ids.shape
    order = np.argsort(ids)
    sorted_ids = ids[order]
    o_all, a_all, p_all, y_all = [], [], [], []
    for r in range(R):
        if int(rel_pred[r]) >= NUM_PROP_PRED:
            continue
        o = rng.integers(0, n, per_relation)
        b = bind_ids[r, o]
        keep = b != FARM_NO_ID
        o, b = o[keep], b[keep]
        a_pos = order[np.searchsorted(sorted_ids, b)]
        o_neg = np.repeat(o, negatives)
        a_neg = rng.integers(0, n - 1, o_neg.size)
        a_neg = a_neg + (a_neg >= o_neg)  # uniform over a != o
        b_neg = np.repeat(a_pos, negatives)
        oo = np.concatenate([o, o_neg])
        aa = np.concatenate([a_pos, a_neg])
        yy = np.concatenate([np.ones(o.size, np.float32), (a_neg == b_neg).astype(np.float32)])
        o_all.append(oo)
        a_all.append(aa)
        p_all.append(np.full(oo.size, int(rel_pred[r]), np.int32))
        y_all.append(yy)
    cat = lambda xs, dt: np.concatenate(xs).astype(dt) if xs else np.zeros(0, dt)
    return cat(o_all, np.int32), cat(a_all, np.int32), cat(p_all, np.int32), cat(y_all, np.float32)


def train(net: ProposalNet, data: list, steps: int, batch: int = 4096, lr: float = 1e-3,
          weight_decay: float = 1e-4, seed: int = 0, log_every: int = 50, stream=None):
    """AdamW steps over shuffled mini-batches of `data` = [(mem, o, a, pred, label), ...].

    Each step draws one scene (round-robin) and a batch of its examples.
    Returns the recorded losses [(step, loss)]."""
    import torch
    rng = np.random.default_rng(seed)
    dev = torch.device("cuda:0")
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    history = []
    batch = min(batch, net.max_batch)
    for step in range(steps):
        mem, o, a, p, y = data[step % len(data)]
        sel = rng.integers(0, o.size, batch)
        up = lambda x: torch.from_numpy(np.ascontiguousarray(x[sel])).to(dev)
        net.step(mem, up(o), up(a), up(p), up(y), lr=lr, weight_decay=weight_decay, update=True, loss_out=loss,
                 stream=stream)
        if step % log_every == 0 or step == steps - 1:
            torch.cuda.synchronize()
            history.append((step, float(loss.item())))
    return history
