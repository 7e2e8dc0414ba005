"""Brute-force joint-binding enumeration for tiny scenes (test infrastructure only).

This is the score *before* the star decomposition: for a candidate target e,
every binding eta of the anchor variables (a_1..a_R) to memory entities other
than e is verified and the best one kept (Appendix "Robust Relational
Retrieval Formulation", soft verification: score(e) is the maximum of
Verify(eta) over bindings with eta(x_star) = e).  Verify aggregates the unary
target score and the induced relational scores with the composite rule of the
Appendix "Retrieval Details", composite-scoring step:

    Verify(eta) = s_sem(e) * ((1 - w) + w * gmean_r( sim(eta(a_r), q_r) * P_r(e, eta(a_r)) ))

Each relation's term folds the anchor's own description match sim(a, q_r)
into the relational score (the anchor's unary predicate and the relation share
the anchor variable).  Pure Python on math.* in double precision; it shares no code
with ``farm_oracle.c`` and costs O(N^(R+1)) -- use N <= 16, R <= 3.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

W = 0.5
CLASS_FACTOR = 0.3
BETWEEN_K = 64


def _unit(v):
    s = math.sqrt(sum(float(x) * float(x) for x in v))
    return [float(x) / s for x in v]


def _sim(u, v):
    return max(0.0, sum(a * b for a, b in zip(u, v)))


def _sigmoid(x):
    if x < 0:  # the same value without overflowing exp(-x)
        e = math.exp(x)
        return e / (1.0 + e)
    return 1.0 / (1.0 + math.exp(-x))


def soft_relation(pred, ci, cj, right, ei=(0.0, 0.0, 0.0), ej=(0.0, 0.0, 0.0)):
    """The ten closed-form soft predicates, written from their definitions
    (ei, ej: full box extents of target and anchor, used by On and Inside)."""
    dx, dy, dz = (float(ci[0]) - float(cj[0]), float(ci[1]) - float(cj[1]), float(ci[2]) - float(cj[2]))
    if pred == 11:  # inside: the target's center within the anchor's box, softly per axis
        v = 1.0
        for k in range(3):
            v *= _sigmoid((float(ej[k]) / 2.0 - abs(float(ci[k]) - float(cj[k]))) / 0.1)
        return v
    if pred == 8:  # on: gate on the horizontal distance (sigma 0.5 m) times a band on the
        # gap between the target's bottom face and the anchor's top face (sigma 0.125 m)
        bottom_i = float(ci[2]) - float(ei[2]) / 2.0
        top_j = float(cj[2]) + float(ej[2]) / 2.0
        gate = math.exp(-(dx * dx + dy * dy) / (2 * 0.5 * 0.5))
        band = math.exp(-((bottom_i - top_j) ** 2) / (2 * 0.125 * 0.125))
        return gate * band
    if pred == 0:  # near: Gaussian on centroid distance, sigma 0.5 m
        return math.exp(-(dx * dx + dy * dy + dz * dz) / (2 * 0.25))
    if pred == 5:  # next to: the same Gaussian with sigma 1 m
        return math.exp(-(dx * dx + dy * dy + dz * dz) / 2.0)
    if pred == 1:  # above: sigmoid of the vertical offset, temperature 0.1 m
        return _sigmoid(dz / 0.1)
    if pred == 2:  # below
        return _sigmoid(-dz / 0.1)
    rx, ry = float(right[0]), float(right[1])
    lateral = dx * rx + dy * ry
    if pred == 4:  # right of
        return _sigmoid(lateral / 0.1)
    if pred == 3:  # left of
        return _sigmoid(-lateral / 0.1)
    # viewing direction: the right axis turned a quarter turn counter-clockwise
    depth = dx * (-ry) + dy * rx
    if pred == 6:  # in front of: nearer the viewer than the anchor
        return _sigmoid(-depth / 0.1)
    if pred == 7:  # behind
        return _sigmoid(depth / 0.1)
    raise ValueError(pred)


def between_relation(ci, c1, c2):
    """Between (ternary): the target's center projects inside the segment
    joining the two anchors' centers (a logistic, 0.1 m, of each margin along
    it) and lies near it (Gaussian, 0.5 m, of the distance to the foot of the
    projection); 0 for coincident anchors."""
    ci, c1, c2 = ([float(v) for v in c] for c in (ci, c1, c2))
    u = [c2[k] - c1[k] for k in range(3)]
    uu = sum(x * x for x in u)
    if uu == 0.0:
        return 0.0
    lam = sum((ci[k] - c1[k]) * u[k] for k in range(3)) / uu  # position along the segment, 0 at c1, 1 at c2
    foot = [c1[k] + lam * u[k] for k in range(3)]
    h2 = sum((ci[k] - foot[k]) ** 2 for k in range(3))
    L = math.sqrt(uu)
    return _sigmoid(lam * L / 0.1) * _sigmoid((1.0 - lam) * L / 0.1) * math.exp(-h2 / (2 * 0.25))


def _solve_and_logdet(M, v):
    """x with M x = v, and log det M, by Gaussian elimination with partial pivoting (M 3x3, positive definite)."""
    A = [list(map(float, M[r])) + [float(v[r])] for r in range(3)]
    logdet = 0.0
    for c in range(3):
        piv = max(range(c, 3), key=lambda r: abs(A[r][c]))
        if piv != c:
            A[c], A[piv] = A[piv], A[c]
        logdet += math.log(abs(A[c][c]))
        for r in range(c + 1, 3):
            f = A[r][c] / A[c][c]
            for k in range(c, 4):
                A[r][k] -= f * A[c][k]
    x = [0.0, 0.0, 0.0]
    for r in (2, 1, 0):
        x[r] = (A[r][3] - sum(A[r][k] * x[k] for k in range(r + 1, 3))) / A[r][r]
    return x, logdet


def _sym(p6):
    a, b, c, d, e, f = (float(v) for v in p6)
    return [[a, b, c], [b, d, e], [c, e, f]]


def hellinger_relation(ci, cov_i, cj, cov_j):
    """Near over entity Gaussians: 1 - H, H^2 = 1 - exp(-D_B) with the Bhattacharyya distance
    D_B = (mu_i - mu_j)^T M^-1 (mu_i - mu_j) / 8 + log(det M / sqrt(det A det B)) / 2, M = (A + B) / 2."""
    A, B = _sym(cov_i), _sym(cov_j)
    M = [[(A[r][k] + B[r][k]) / 2.0 for k in range(3)] for r in range(3)]
    dmu = [float(ci[k]) - float(cj[k]) for k in range(3)]
    x, ld_m = _solve_and_logdet(M, dmu)
    _, ld_a = _solve_and_logdet(A, [0.0, 0.0, 0.0])
    _, ld_b = _solve_and_logdet(B, [0.0, 0.0, 0.0])
    db = sum(dmu[k] * x[k] for k in range(3)) / 8.0 + 0.5 * (ld_m - 0.5 * (ld_a + ld_b))
    return 1.0 - math.sqrt(max(0.0, 1.0 - math.exp(-db)))


def view_relation(pred, view_i, ci, cj):
    """LeftOf / RightOf / InFrontOf / Behind (15..18) in target i's stored view: a pinhole camera at
    view_i[0:3] with right, down and forward axes view_i[3:6], [6:9], [9:12]; horizontal image-plane
    coordinate u = (w . right) / (w . forward), depth w . forward, w the offset from the camera.  Both
    objects must be in the view (depth >= 0.1 m, |x| <= depth, |y| <= 0.75 depth), else 0."""
    v = [float(x) for x in view_i]
    pos, right, down, fwd = v[0:3], v[3:6], v[6:9], v[9:12]

    def cam(c):
        w = [float(c[k]) - pos[k] for k in range(3)]
        return (sum(w[k] * right[k] for k in range(3)), sum(w[k] * down[k] for k in range(3)),
                sum(w[k] * fwd[k] for k in range(3)))

    (xi, yi, zi), (xj, yj, zj) = cam(ci), cam(cj)
    for x, y, z in ((xi, yi, zi), (xj, yj, zj)):
        if not (z >= 0.1 and abs(x) <= z and abs(y) <= 0.75 * z):
            return 0.0
    ui, uj = xi / zi, xj / zj
    if pred == 15:
        return _sigmoid((uj - ui) / 0.05)
    if pred == 16:
        return _sigmoid((ui - uj) / 0.05)
    if pred == 17:  # in front of: nearer the camera
        return _sigmoid((zj - zi) / 0.1)
    if pred == 18:
        return _sigmoid((zi - zj) / 0.1)
    raise ValueError(pred)


def rank_relation(pred, scene, tcls, i, j):
    """Closest (9) / Farthest (10): 1 / (|rank - r*| + 1), the rank of target i
    among the query's candidates (objects of class tcls; all objects without a
    class) by Euclidean distance to anchor j, nearer first, equal distances by
    id; r* = 1 for Closest and the last rank for Farthest."""
    c = [[float(v) for v in row] for row in scene.center]

    def dist(a, b):
        return math.sqrt(sum((c[a][k] - c[b][k]) ** 2 for k in range(3)))

    dij = dist(i, j)
    nearer = m = 0
    for k in range(scene.desc.shape[0]):
        if k in (i, j):
            continue
        if tcls >= 0 and scene.cls is not None and int(scene.cls[k]) != tcls:
            continue
        m += 1
        dk = dist(k, j)
        if dk < dij or (dk == dij and int(scene.ids[k]) < int(scene.ids[i])):
            nearer += 1
    rank = nearer + 1
    rstar = 1 if pred == 9 else m + 1
    return 1.0 / (abs(rank - rstar) + 1)


def brute_scores(scene, qb, sims=None):
    """Scores [q][n] by enumerating all anchor bindings (list of lists of floats).  ``sims`` =
    (sem [q][n], asim [r_tot][n]) replaces the clamped cosines as the unary scores (sem with
    the class factor already applied)."""
    n = scene.desc.shape[0]
    units = [_unit(scene.desc[i]) for i in range(n)]
    out = []
    for k in range(qb.target.shape[0]):
        kq = k  # (k is reused by the binding loop below)
        qt = _unit(qb.target[k])
        tcls = int(qb.target_cls[k]) if qb.target_cls is not None else -1
        a0, a1 = int(qb.rel_off[k]), int(qb.rel_off[k + 1])
        rels = [(int(qb.rel_pred[r]), _unit(qb.rel_anchor[r])) for r in range(a0, a1)]
        if sims is not None:  # unary scores given: the anchor "vector" is the row index
            rels = [(int(qb.rel_pred[r]), r) for r in range(a0, a1)]
        if sims is None:
            asim_of = lambda j, qr: _sim(units[j], qr)
        else:
            asim_of = lambda j, r: float(sims[1][r][j])
        row = []
        for e in range(n):
            kappa = 1.0
            if tcls >= 0 and scene.cls is not None and int(scene.cls[e]) >= 0 and int(scene.cls[e]) != tcls:
                kappa = CLASS_FACTOR
            s_sem = kappa * _sim(units[e], qt) if sims is None else float(sims[0][kq][e])
            if not rels:
                row.append(s_sem)
                continue
            others = [j for j in range(n) if j != e]
            best = None
            if not others:
                best = s_sem * (1 - W)
            # predicate invocations: a Between (12) takes its slot's and the next
            # slot's (13) anchor variables together and counts once; those two
            # variables range over their candidate sets (the 64 anchors of
            # largest similarity, ties by smaller id)
            n_inv = sum(1 for pred, _ in rels if pred != 13)
            domains = []
            for pred, qr in rels:
                if pred in (12, 13):
                    order = sorted(range(n), key=lambda j: (-asim_of(j, qr), int(scene.ids[j])))
                    cand = set(order[:BETWEEN_K])
                    domains.append([j for j in others if j in cand])
                else:
                    domains.append(others)
            for binding in itertools.product(*domains):
                prod = 1.0
                for k, ((pred, qr), j) in enumerate(zip(rels, binding)):
                    if pred == 13:
                        continue
                    if pred == 12:
                        j2 = binding[k + 1]
                        pv = 0.0 if j2 == j else between_relation(scene.center[e], scene.center[j], scene.center[j2])
                        prod *= asim_of(j, qr) * asim_of(j2, rels[k + 1][1]) * pv
                        continue
                    if pred in (9, 10):
                        pv = rank_relation(pred, scene, tcls, e, j)
                    elif pred == 14:
                        pv = hellinger_relation(scene.center[e], scene.cov[e], scene.center[j], scene.cov[j])
                    elif 15 <= pred <= 18:
                        pv = view_relation(pred, scene.view[e], scene.center[e], scene.center[j])
                    else:
                        pv = soft_relation(pred, scene.center[e], scene.center[j], scene.view_right,
                                           scene.extent[e], scene.extent[j])
                    prod *= asim_of(j, qr) * pv
                v = s_sem * ((1 - W) + W * prod ** (1.0 / n_inv))
                if best is None or v > best:
                    best = v
            row.append(best)
        out.append(row)
    return out
