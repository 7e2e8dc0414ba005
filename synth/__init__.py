"""Seeded synthetic scenes and query batches for the relational retrieval path.

This module only draws random inputs. It holds none of the scoring arithmetic
(no similarity, no predicate, no composite): both the CPU oracle and the GPU
path consume what it produces, and neither imports the other.

A scene stands in for the object-level memory of the paper (Section 2.2,
"Representation"): per object a retrieval descriptor, a 3-D axis-aligned box
(center, full extents), a unique object id, a category id, and one viewer frame
per scene (the right-pointing unit vector of a virtual viewer in the ground
plane). A query batch stands in for the parsed query graph (Section 2.3,
"Executable query specification"): a target embedding, a target class and an
ordered list of (predicate, anchor embedding) relations, stored in CSR form.

The paper's benchmarks (ReferIt3D/ScanNet, IRef-VLA/HM3D, FARM-Scenes) are not
available; the configurations below replace them with synthetic scenes whose
extents echo the paper's scene-scale range (a room, a two-floor office, a
15,000 m^2 outdoor/indoor site, cf. the FARM-Scenes data card).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Predicate ids, in the order the C ABI uses.
NEAR, ABOVE, BELOW, LEFT_OF, RIGHT_OF = 0, 1, 2, 3, 4
NEXT_TO, IN_FRONT_OF, BEHIND, ON = 5, 6, 7, 8
CLOSEST, FARTHEST, INSIDE = 9, 10, 11
BETWEEN, AND = 12, 13                       # ternary Between: its slot, then its second anchor's slot
# over entity Gaussians (Hellinger Near) and per-object stored views (image-plane / depth offsets)
NEAR_H, LEFT_OF_V, RIGHT_OF_V, IN_FRONT_OF_V, BEHIND_V = 14, 15, 16, 17, 18
VIEW_PREDS = (LEFT_OF_V, RIGHT_OF_V, IN_FRONT_OF_V, BEHIND_V)
GEOMETRY_PREDS = (NEAR_H,) + VIEW_PREDS
ALL_PREDS = tuple(range(9))                 # the pairwise predicates with learned anchor lists
RANK_PREDS = (CLOSEST, FARTHEST)            # rank within the query's candidate set
EVERY_PRED = ALL_PREDS + RANK_PREDS + (INSIDE,)
DEFAULT_PREDS = (NEAR, ABOVE, BELOW, LEFT_OF, RIGHT_OF)  # the pool query batches draw from by default
PRED_NAMES = ("near", "above", "below", "left_of", "right_of", "next_to", "in_front_of", "behind", "on", "closest",
              "farthest", "inside", "between", "and", "near_hellinger", "left_of_view", "right_of_view",
              "in_front_of_view", "behind_view")


@dataclasses.dataclass
class Scene:
    desc: np.ndarray        # [n, d] float32, unnormalised rows
    center: np.ndarray      # [n, 3] float32, metres, z up
    extent: np.ndarray      # [n, 3] float32, full side lengths (> 0)
    ids: np.ndarray         # [n] uint32, unique, never 0xFFFFFFFF
    cls: np.ndarray         # [n] int32, category id (>= 0)
    view_right: np.ndarray  # [2] float32, viewer right vector (x, y)
    centroids: np.ndarray   # [C, d] float32, category centroids (unit rows)
    cov: np.ndarray | None = None   # [n, 6] float32 entity covariances (xx, xy, xz, yy, yz, zz), or None
    view: np.ndarray | None = None  # [n, 12] float32 stored views: camera center, then its right, down and
    #                                 forward axes (the rows of the world-to-camera rotation), or None

    @property
    def n(self) -> int:
        return int(self.desc.shape[0])

    @property
    def d(self) -> int:
        return int(self.desc.shape[1])


@dataclasses.dataclass
class QueryBatch:
    target: np.ndarray      # [q, d] float32
    target_cls: np.ndarray  # [q] int32 (-1 = no class)
    rel_off: np.ndarray     # [q + 1] int32, CSR offsets into the relation arrays
    rel_pred: np.ndarray    # [r_tot] int32 predicate ids
    rel_anchor: np.ndarray  # [r_tot, d] float32
    planted: np.ndarray     # [q] int64 index of the object the query was drawn from (diagnostic only)

    @property
    def q(self) -> int:
        return int(self.target.shape[0])

    @property
    def r_tot(self) -> int:
        return int(self.rel_pred.shape[0])

    def subset(self, rows) -> "QueryBatch":
        rows = np.asarray(rows, dtype=np.int64)
        offs, preds, anchors = [0], [], []
        for r in rows:
            a, b = int(self.rel_off[r]), int(self.rel_off[r + 1])
            preds.append(self.rel_pred[a:b])
            anchors.append(self.rel_anchor[a:b])
            offs.append(offs[-1] + (b - a))
        d = self.target.shape[1]
        return QueryBatch(
            target=np.ascontiguousarray(self.target[rows]),
            target_cls=np.ascontiguousarray(self.target_cls[rows]),
            rel_off=np.asarray(offs, dtype=np.int32),
            rel_pred=np.ascontiguousarray(np.concatenate(preds) if preds else np.zeros(0, np.int32)).astype(np.int32),
            rel_anchor=np.ascontiguousarray(np.concatenate(anchors) if anchors else np.zeros((0, d), np.float32)).astype(np.float32),
            planted=np.ascontiguousarray(self.planted[rows]),
        )


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    seed: int
    n: int
    d: int
    n_cat: int
    noise: float            # descriptor noise norm (per-component std = noise / sqrt(d))
    layout: str             # "uniform_room" | "rooms_two_floor" | "site_mix"
    q: int
    r_min: int
    r_max: int
    k: int = 10


TINY = Config("tiny", 0, 64, 512, 16, 0.15, "uniform_room", 8, 2, 2)
MID = Config("mid", 1, 2000, 1024, 200, 0.10, "rooms_two_floor", 256, 1, 3)
PRECISION = Config("precision", 2, 20000, 1152, 500, 0.10, "site_mix", 4096, 1, 4)
CONFIGS = {c.name: c for c in (TINY, MID, PRECISION)}


def _unit_rows(x: np.ndarray) -> np.ndarray:
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def _noisy(rng: np.random.Generator, base: np.ndarray, noise: float) -> np.ndarray:
    d = base.shape[-1]
    eps = rng.standard_normal(base.shape) * (noise / math.sqrt(d))
    return _unit_rows(np.atleast_2d(base + eps))


def _centers(rng: np.random.Generator, n: int, layout: str) -> np.ndarray:
    if layout == "uniform_room":
        return rng.uniform([0.0, 0.0, 0.0], [10.0, 10.0, 3.0], size=(n, 3))
    if layout == "rooms_two_floor":
        n_rooms = 20
        room_xy = rng.uniform(0.0, 60.0, size=(n_rooms, 2))
        room_base = rng.choice([0.0, 3.0], size=n_rooms)
        room = rng.integers(0, n_rooms, size=n)
        xy = room_xy[room] + rng.normal(0.0, 2.0, size=(n, 2))
        z = room_base[room] + rng.uniform(0.0, 3.0, size=n)
        return np.column_stack([xy, z])
    if layout == "site_mix":
        # Half indoor (40 rooms on three floors spanning 0-10 m), half outdoor
        # (uniform over the 150 x 100 m footprint, objects up to 2 m high).
        n_in = n // 2
        n_out = n - n_in
        n_rooms = 40
        floor_h = 10.0 / 3.0
        room_xy = rng.uniform([0.0, 0.0], [150.0, 100.0], size=(n_rooms, 2))
        room_base = rng.integers(0, 3, size=n_rooms) * floor_h
        room = rng.integers(0, n_rooms, size=n_in)
        xy_in = room_xy[room] + rng.normal(0.0, 2.0, size=(n_in, 2))
        z_in = room_base[room] + rng.uniform(0.0, floor_h, size=n_in)
        xy_out = rng.uniform([0.0, 0.0], [150.0, 100.0], size=(n_out, 2))
        z_out = rng.uniform(0.0, 2.0, size=n_out)
        c = np.concatenate([np.column_stack([xy_in, z_in]), np.column_stack([xy_out, z_out])])
        return c[rng.permutation(n)]
    raise ValueError(f"unknown layout {layout!r}")


def make_scene(cfg: Config, seed: int | None = None, n: int | None = None) -> Scene:
    """Draw one scene. ``seed``/``n`` override the config's values."""
    seed = cfg.seed if seed is None else seed
    n = cfg.n if n is None else n
    rng = np.random.default_rng([seed, 0x5CE9E])
    centroids = _unit_rows(rng.standard_normal((cfg.n_cat, cfg.d)))
    cls = rng.integers(0, cfg.n_cat, size=n).astype(np.int32)
    desc = _noisy(rng, centroids[cls], cfg.noise) if n else np.zeros((0, cfg.d))
    center = _centers(rng, n, cfg.layout)
    extent = np.exp(rng.uniform(math.log(0.1), math.log(2.0), size=(n, 3)))
    # Object ids are unique but unrelated to the storage order, so that the
    # id tie-break is exercised independently of the index order.
    ids = (rng.choice(16 * max(n, 1), size=n, replace=False) + 1).astype(np.uint32)
    yaw = rng.uniform(0.0, 2.0 * math.pi)
    view_right = np.array([math.sin(yaw), -math.cos(yaw)], dtype=np.float32)
    return Scene(
        desc=np.ascontiguousarray(desc, dtype=np.float32),
        center=np.ascontiguousarray(center, dtype=np.float32),
        extent=np.ascontiguousarray(extent, dtype=np.float32),
        ids=ids,
        cls=cls,
        view_right=view_right,
        centroids=centroids.astype(np.float32),
    )


def add_entity_geometry(scene: Scene, seed: int = 0) -> Scene:
    """The scene with an entity Gaussian and one stored view per object.

    Gaussian: mean = the box center; covariance = the second moment of a
    uniform distribution over the box (e^2 / 12 per axis), each axis scaled by
    a factor in [0.8, 1.25] and turned by a random yaw.  View: a camera 0.8 to
    3.0 m from the object horizontally (the viewpoint-distance range of the
    paper's HM3D trajectories), 0.2 to 0.8 m above its center, looking at it
    with a level horizon.
    """
    rng = np.random.default_rng([seed, 0x6A55])
    n = scene.n
    e = scene.extent.astype(np.float64)
    var = (e * e / 12.0) * rng.uniform(0.8, 1.25, size=(n, 3))
    yaw = rng.uniform(0.0, math.pi, size=n)
    cov = np.zeros((n, 6))
    for i in range(n):
        c, s_ = math.cos(yaw[i]), math.sin(yaw[i])
        R = np.array([[c, -s_, 0.0], [s_, c, 0.0], [0.0, 0.0, 1.0]])
        S = R @ np.diag(var[i]) @ R.T
        cov[i] = [S[0, 0], S[0, 1], S[0, 2], S[1, 1], S[1, 2], S[2, 2]]
    c64 = scene.center.astype(np.float64)
    dist = rng.uniform(0.8, 3.0, size=n)
    az = rng.uniform(0.0, 2.0 * math.pi, size=n)
    up = rng.uniform(0.2, 0.8, size=n)
    view = np.zeros((n, 12))
    for i in range(n):
        pos = c64[i] + np.array([dist[i] * math.cos(az[i]), dist[i] * math.sin(az[i]), up[i]])
        fwd = c64[i] - pos
        fwd /= np.linalg.norm(fwd)
        right = np.cross(fwd, [0.0, 0.0, 1.0])
        right /= np.linalg.norm(right)
        down = np.cross(fwd, right)
        view[i] = np.concatenate([pos, right, down, fwd])
    return dataclasses.replace(scene, cov=np.ascontiguousarray(cov, dtype=np.float32),
                               view=np.ascontiguousarray(view, dtype=np.float32))


def _camera(scene: Scene, o: int, c64: np.ndarray) -> np.ndarray:
    """Camera-frame coordinates of every center in object o's stored view."""
    v = scene.view[o].astype(np.float64)
    return (c64 - v[:3]) @ v[3:].reshape(3, 3).T


def _plant_anchor(rng, scene: Scene, o: int, pred: int, c64: np.ndarray, r64: np.ndarray) -> int:
    """Pick the anchor object for a planted relation by a geometric rule.

    The rule only decides which object the query talks about (the nearest
    object lying clearly on the named side of the target); it is not the
    predicate's soft score, which the scorers compute.
    """
    d = c64 - c64[o]
    dist = np.sqrt((d * d).sum(axis=1))
    dist[o] = np.inf
    if pred in (NEAR, NEXT_TO, CLOSEST, INSIDE, NEAR_H):
        ok = np.isfinite(dist)
    elif pred in VIEW_PREDS and scene.view is not None:
        # in o's stored view: both in front of the camera, the anchor on the named side
        # (0.1 of the image plane) or at the named depth (0.3 m)
        xc = _camera(scene, o, c64)
        vis = (xc[:, 2] > 0.3) & (np.abs(xc[:, 0]) < 0.9 * xc[:, 2]) & (np.abs(xc[:, 1]) < 0.7 * xc[:, 2])
        u = xc[:, 0] / np.where(xc[:, 2] > 0, xc[:, 2], 1.0)
        side = {LEFT_OF_V: u - u[o], RIGHT_OF_V: u[o] - u, IN_FRONT_OF_V: (xc[:, 2] - xc[o, 2]) / 3.0,
                BEHIND_V: (xc[o, 2] - xc[:, 2]) / 3.0}[pred]
        ok = vis & (side > 0.1)
    elif pred == FARTHEST:
        ok = np.isfinite(dist)
        dist = np.where(ok, -dist, np.inf)  # the farthest object
    elif pred == ON:
        # the horizontally nearest object whose center lies at least 0.3 m lower
        ok = -d[:, 2] > 0.3
        dist = np.sqrt(d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1])
        dist[o] = np.inf
    elif pred in (ABOVE, BELOW):
        # Target above the anchor: anchor lies at least 0.3 m lower.
        side = -d[:, 2] if pred == ABOVE else d[:, 2]
        ok = side > 0.3
    elif pred in (LEFT_OF, RIGHT_OF):
        lateral = -(d[:, 0] * r64[0] + d[:, 1] * r64[1])  # (target - anchor) . right
        side = lateral if pred == RIGHT_OF else -lateral
        ok = side > 0.3
    else:
        # viewing direction (-r_y, r_x); in front = the anchor lies at least 0.3 m farther away
        farther = d[:, 0] * -r64[1] + d[:, 1] * r64[0]  # (anchor - target) . forward
        side = farther if pred == IN_FRONT_OF else -farther
        ok = side > 0.3
    ok &= np.isfinite(dist)
    if not ok.any():
        return -1
    cand = np.flatnonzero(ok)
    return int(cand[np.argmin(dist[cand])])


def make_queries(cfg: Config, scene: Scene, seed: int | None = None, q: int | None = None,
                 r_min: int | None = None, r_max: int | None = None,
                 with_class: bool = True, preds=None) -> QueryBatch:
    """Draw a query batch against ``scene``.

    Each query picks a planted target object, uses a noisy copy of its category
    centroid as the target embedding, and draws R relations; each relation has
    a uniformly drawn predicate and the anchor embedding of a noisy centroid of
    a geometrically suitable anchor object's category.  ``preds`` lists the
    predicate ids to draw from (default: ``DEFAULT_PREDS``, Near..RightOf).
    """
    pool = DEFAULT_PREDS if preds is None else tuple(int(p) for p in preds)
    seed = cfg.seed if seed is None else seed
    q = cfg.q if q is None else q
    r_min = cfg.r_min if r_min is None else r_min
    r_max = cfg.r_max if r_max is None else r_max
    rng = np.random.default_rng([seed, 0x9E27])
    n, d = scene.n, scene.d
    c64 = scene.center.astype(np.float64)
    r64 = scene.view_right.astype(np.float64)
    targets, tcls, offs, preds, anchors, planted = [], [], [0], [], [], []
    for _ in range(q):
        o = int(rng.integers(0, n))
        k = int(scene.cls[o])
        targets.append(_noisy(rng, scene.centroids[k][None].astype(np.float64), cfg.noise)[0])
        tcls.append(k if with_class else -1)
        planted.append(o)
        r = int(rng.integers(r_min, r_max + 1))
        for _ in range(r):
            for _attempt in range(16):
                p = pool[int(rng.integers(0, len(pool)))]
                j = _plant_anchor(rng, scene, o, p, c64, r64) if n > 1 else -1
                if j >= 0:
                    break
            if j < 0:  # degenerate scene: any object's category
                j = int(rng.integers(0, n))
            preds.append(p)
            anchors.append(_noisy(rng, scene.centroids[int(scene.cls[j])][None].astype(np.float64), cfg.noise)[0])
        offs.append(len(preds))
    return QueryBatch(
        target=np.ascontiguousarray(np.asarray(targets, dtype=np.float32).reshape(q, d)),
        target_cls=np.asarray(tcls, dtype=np.int32),
        rel_off=np.asarray(offs, dtype=np.int32),
        rel_pred=np.asarray(preds, dtype=np.int32),
        rel_anchor=np.ascontiguousarray(np.asarray(anchors, dtype=np.float32).reshape(len(preds), d)),
        planted=np.asarray(planted, dtype=np.int64),
    )


def add_between(cfg: Config, scene: Scene, qb: QueryBatch, seed: int, every: int = 1) -> QueryBatch:
    """Append one Between invocation (two slots: BETWEEN, then AND) to every
    ``every``-th query that has room (R + 2 <= 8).  Its anchors are planted by
    a geometric rule around the query's planted target o: the object nearest
    to o, then the object nearest to o on the far side of o from it (positive
    offset along the direction from the first anchor to o); their embeddings
    are noisy centroids of their categories."""
    rng = np.random.default_rng([seed, 0xB7])
    c64 = scene.center.astype(np.float64)
    offs, preds, anchors = [0], [], []
    d = scene.d
    for k in range(qb.q):
        a, b = int(qb.rel_off[k]), int(qb.rel_off[k + 1])
        preds += [int(v) for v in qb.rel_pred[a:b]]
        anchors += list(qb.rel_anchor[a:b])
        o = int(qb.planted[k])
        if k % every == 0 and b - a + 2 <= 8 and scene.n >= 3:
            dist = np.sqrt(((c64 - c64[o]) ** 2).sum(axis=1))
            dist[o] = np.inf
            j1 = int(np.argmin(dist))
            axis = c64[o] - c64[j1]
            far = (c64 - c64[o]) @ axis > 0
            far[[o, j1]] = False
            j2 = int(np.flatnonzero(far)[np.argmin(dist[far])]) if far.any() else int(np.argsort(dist)[1])
            preds += [BETWEEN, AND]
            for j in (j1, j2):
                anchors.append(_noisy(rng, scene.centroids[int(scene.cls[j])][None].astype(np.float64), cfg.noise)[0])
        offs.append(len(preds))
    return QueryBatch(
        target=qb.target, target_cls=qb.target_cls, rel_off=np.asarray(offs, dtype=np.int32),
        rel_pred=np.asarray(preds, dtype=np.int32),
        rel_anchor=np.ascontiguousarray(np.asarray(anchors, dtype=np.float32).reshape(len(preds), d)),
        planted=qb.planted)


def add_embedding_spaces(cfg: Config, scene: Scene, qb: QueryBatch, dims=(512, 768), seed: int = 0):
    """Further per-entity embedding spaces and the batch's query vectors in them, standing in for
    the several retrieval embeddings stored per entity (a caption-text and two image embeddings).

    Space s has class centroids of its own; an entity's embedding is a noisy copy of its class's
    centroid.  The targets' vectors are noisy centroids of the planted object's class; an anchor's
    vector is a noisy centroid of the class whose descriptor-space centroid its descriptor-space
    vector lies closest to (the class it was drawn from).  Returns (spaces [n, d_s] list,
    target vectors [q, d_s] list, anchor vectors [r_tot, d_s] list)."""
    rng = np.random.default_rng([seed, 0xE3B5])
    anchor_cls = (np.asarray(qb.rel_anchor, np.float64) @ scene.centroids.astype(np.float64).T).argmax(axis=1) \
        if qb.r_tot else np.zeros(0, np.int64)
    target_cls = scene.cls[np.asarray(qb.planted, np.int64)]
    spaces, tv, av = [], [], []
    for d in dims:
        cent = _unit_rows(rng.standard_normal((scene.centroids.shape[0], d)))
        spaces.append(np.ascontiguousarray(_noisy(rng, cent[scene.cls], cfg.noise), np.float32))
        tv.append(np.ascontiguousarray(_noisy(rng, cent[target_cls], cfg.noise), np.float32))
        av.append(np.ascontiguousarray(_noisy(rng, cent[anchor_cls], cfg.noise), np.float32).reshape(qb.r_tot, d))
    return spaces, tv, av


def make_workload(name: str, **kw):
    cfg = CONFIGS[name]
    scene = make_scene(cfg, n=kw.pop("n", None), seed=kw.pop("scene_seed", None))
    queries = make_queries(cfg, scene, **kw)
    return cfg, scene, queries
