"""Multi-channel reciprocal-rank fusion of the unary scores, FP64 (test infrastructure only).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: it shares no code with the GPU library.

Candidate retrieval (Appendix "Retrieval Details", step 3): the whole candidate pool is ranked
by reciprocal-rank fusion over several query channels -- each channel a query vector in one of
the entity embedding spaces -- where channel c contributes w_c / (mu + rank_c(i)), mu = 5; the
fused score is the entity's target similarity s_sem, and the landmarks of the relations are
retrieved analogously (Section "Robust Relational Object Retrieval", implementation paragraph:
unary scores by reciprocal-rank fusion over the stored retrieval embeddings).

Readings (the paper gives the formula, not these details):
  * rank_c(i) = 1 + #{j != i : cos_c(j) > cos_c(i), or equal and id_j < id_i}: the pool ordered
    by the cosine of the channel's query vector with each entity's embedding in the channel's
    space, largest first, equal cosines by smaller id;
  * the fused score is divided by its largest possible value sum_c w_c / (mu + 1), so that it
    lies in (0, 1] like the other unary scores (1 for the first of every channel);
  * target rows then take the soft class factor (0.3 for a known, different class); relation
    rows use the same channels with the anchor description's vectors.
"""
from __future__ import annotations

import numpy as np

MU = 5.0


def _unit(a):
    a = np.asarray(a, np.float64)
    return a / np.linalg.norm(a, axis=-1, keepdims=True)


def channel_ranks(cos, ids, mode: int = 0, eps: float = 0.0):
    """Ranks [rows, n] of every entity per row of cosines [rows, n] (1 = largest; equal cosines by
    smaller id).  mode -1 / +1: the smallest / largest rank the entity can take when cosines within
    ``eps`` of its own may fall on either side (an implementation whose cosines are within eps)."""
    cos = np.asarray(cos, np.float64)
    ids = np.asarray(ids, np.int64)
    rows, n = cos.shape
    out = np.zeros((rows, n), np.int64)
    for r in range(rows):
        c = cos[r]
        if mode == 0:
            order = np.lexsort((ids, -c))        # cosine descending, then id ascending
            out[r, order] = np.arange(1, n + 1)
        else:
            s = np.sort(c)
            if mode < 0:   # only the surely larger ones come first
                out[r] = 1 + (n - np.searchsorted(s, c + eps, side="right"))
            else:          # every possibly larger one comes first (the entity itself excluded)
                out[r] = (n - np.searchsorted(s, c - eps, side="left"))
    return out


def fused(spaces, ids, channels, rows: str, mode: int = 0, eps: float = 0.0):
    """Fused score [rows, n] of one kind of row ("target" or "anchor").
    spaces: list of [n, d_s] embedding tables; channels: list of (space, weight, vectors [rows, d_s])."""
    total = sum(float(w) for _, w, _ in channels)
    out = None
    for s_idx, w, vec in channels:
        cos = _unit(vec) @ _unit(spaces[s_idx]).T
        # the largest fused score comes with the smallest rank
        rk = channel_ranks(cos, ids, -mode, eps)
        part = float(w) / (MU + rk)
        out = part if out is None else out + part
    return out / (total / (MU + 1.0))


def similarities(scene, spaces, target_channels, anchor_channels, target_cls, mode: int = 0, eps: float = 0.0):
    """(s_sem [q, n] with the class factor, relation rows sim [r_tot, n]) for the oracle's scorer.
    mode -1 / +1 with eps: the lowest / highest values the tie-aware ranks allow."""
    ids = scene.ids
    sem = fused(spaces, ids, target_channels, "target", mode, eps)
    if scene.cls is not None:
        tc = np.asarray(target_cls, np.int64)[:, None]
        oc = np.asarray(scene.cls, np.int64)[None, :]
        kappa = np.where((tc >= 0) & (oc >= 0) & (tc != oc), 0.3, 1.0)
        sem = sem * kappa
    if anchor_channels and anchor_channels[0][2].shape[0]:
        asim = fused(spaces, ids, anchor_channels, "anchor", mode, eps)
    else:
        asim = np.zeros((0, len(ids)))
    return sem, asim
