"""Synthetic input generators: reproducibility and the statistics each
configuration promises (CPU only).

The generators stand in for the paper's scenes and parsed queries
(Section 2.2 "Representation", Section 2.3 "Executable query specification");
both the oracle and the GPU path consume them, so a drift here would silently
change every parity case and every bench number.
"""
import hashlib

import numpy as np
import pytest

import synth


def _digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def _scene_arrays(s):
    return (s.desc, s.center, s.extent, s.ids, s.cls, s.view_right, s.centroids)


def _query_arrays(qb):
    return (qb.target, qb.target_cls, qb.rel_off, qb.rel_pred, qb.rel_anchor, qb.planted)


@pytest.mark.parametrize("name", ["tiny", "mid"])
def test_same_seed_is_byte_identical(name):
    cfg = synth.CONFIGS[name]
    a = synth.make_scene(cfg)
    b = synth.make_scene(cfg)
    assert _digest(*_scene_arrays(a)) == _digest(*_scene_arrays(b))
    qa = synth.make_queries(cfg, a, q=32)
    qb = synth.make_queries(cfg, b, q=32)
    assert _digest(*_query_arrays(qa)) == _digest(*_query_arrays(qb))


def test_other_seed_differs():
    cfg = synth.TINY
    a = synth.make_scene(cfg, seed=0)
    b = synth.make_scene(cfg, seed=1)
    assert not np.array_equal(a.desc, b.desc)
    assert not np.array_equal(a.center, b.center)
    qa = synth.make_queries(cfg, a, seed=0)
    qb = synth.make_queries(cfg, a, seed=1)
    assert not np.array_equal(qa.target, qb.target)


def test_scene_and_query_streams_are_independent():
    """Changing the query seed leaves the scene untouched and vice versa: the
    two use separate generator streams."""
    cfg = synth.MID
    s0 = synth.make_scene(cfg)
    synth.make_queries(cfg, s0, seed=123, q=8)
    s1 = synth.make_scene(cfg)
    assert _digest(*_scene_arrays(s0)) == _digest(*_scene_arrays(s1))


_BOUNDS = {
    "uniform_room": ((0.0, 0.0, 0.0), (10.0, 10.0, 3.0)),
    # room centres in [0, 60]^2 with N(0, 2 m) scatter: 6 sigma margin
    "rooms_two_floor": ((-12.0, -12.0, 0.0), (72.0, 72.0, 6.0)),
    "site_mix": ((-12.0, -12.0, 0.0), (162.0, 112.0, 10.0)),
}


@pytest.mark.parametrize("name", ["tiny", "mid", "precision"])
def test_scene_statistics_match_config(name):
    cfg = synth.CONFIGS[name]
    n = min(cfg.n, 4000)
    s = synth.make_scene(cfg, n=n)
    assert s.desc.shape == (n, cfg.d) and s.desc.dtype == np.float32
    assert s.center.shape == (n, 3) and s.extent.shape == (n, 3)
    # descriptors: unit rows, each close to its category centroid
    np.testing.assert_allclose(np.linalg.norm(s.desc, axis=1), 1.0, atol=1e-5)
    cos = np.einsum("nd,nd->n", s.desc.astype(np.float64), s.centroids[s.cls].astype(np.float64))
    expect = 1.0 / np.sqrt(1.0 + cfg.noise ** 2)
    assert abs(cos.mean() - expect) < 0.01
    # categories in range and (at these sizes) most of them used
    assert s.cls.min() >= 0 and s.cls.max() < cfg.n_cat
    assert len(np.unique(s.cls)) >= min(cfg.n_cat, n) * 0.6
    # extents log-uniform in [0.1, 2] m
    assert s.extent.min() >= 0.1 - 1e-6 and s.extent.max() <= 2.0 + 1e-6
    lg = np.log(s.extent.astype(np.float64))
    assert abs(lg.mean() - 0.5 * (np.log(0.1) + np.log(2.0))) < 0.05
    # centres inside the layout's footprint
    lo, hi = _BOUNDS[cfg.layout]
    assert (s.center >= np.asarray(lo, np.float32)).all()
    assert (s.center <= np.asarray(hi, np.float32)).all()
    # ids unique, never 0 and never the empty-slot sentinel
    assert len(np.unique(s.ids)) == n
    assert s.ids.min() >= 1 and s.ids.max() < 0xFFFFFFFF
    # viewer right vector lies in the ground plane with unit length
    assert abs(float(np.hypot(*s.view_right.astype(np.float64))) - 1.0) < 1e-6


def test_site_mix_is_half_indoor_half_outdoor():
    """The site layout stands in for a mixed indoor/outdoor site: the outdoor
    half sits below 2 m, the indoor half spans three floors up to 10 m."""
    cfg = synth.PRECISION
    s = synth.make_scene(cfg, n=4000)
    z = s.center[:, 2]
    assert (z > 2.0).mean() > 0.25          # indoor objects on the upper floors
    assert (z <= 2.0).mean() > 0.5          # every outdoor object plus the ground floor's lower part
    assert np.ptp(s.center[:, 0]) > 100.0   # spans the 150 m footprint


@pytest.mark.parametrize("name", ["tiny", "mid", "precision"])
def test_query_statistics_match_config(name):
    cfg = synth.CONFIGS[name]
    s = synth.make_scene(cfg, n=min(cfg.n, 3000))
    qb = synth.make_queries(cfg, s, q=96)
    counts = np.diff(qb.rel_off)
    assert qb.rel_off[0] == 0 and qb.rel_off[-1] == qb.r_tot
    assert counts.min() >= cfg.r_min and counts.max() <= cfg.r_max
    assert set(np.unique(qb.rel_pred)) <= set(synth.DEFAULT_PREDS)
    np.testing.assert_allclose(np.linalg.norm(qb.target, axis=1), 1.0, atol=1e-5)
    np.testing.assert_allclose(np.linalg.norm(qb.rel_anchor, axis=1), 1.0, atol=1e-5)
    # the target class is the planted object's category
    np.testing.assert_array_equal(qb.target_cls, s.cls[qb.planted])
    no_cls = synth.make_queries(cfg, s, q=8, with_class=False)
    assert (no_cls.target_cls == -1).all()


def test_predicate_pool_and_planting_rule():
    """With the full pool all nine predicates appear, and every planted
    anchor category belongs to an object that lies on the named side of the
    target (so the query describes something true of the scene)."""
    cfg = synth.MID
    s = synth.make_scene(cfg)
    qb = synth.make_queries(cfg, s, q=400, preds=synth.ALL_PREDS)
    assert set(np.unique(qb.rel_pred)) == set(synth.ALL_PREDS)
    c = s.center.astype(np.float64)
    r = s.view_right.astype(np.float64)
    fwd = np.array([-r[1], r[0]])
    for qi in range(qb.q):
        o = int(qb.planted[qi])
        for j in range(qb.rel_off[qi], qb.rel_off[qi + 1]):
            p = int(qb.rel_pred[j])
            d = c - c[o]
            if p in (synth.NEAR, synth.NEXT_TO):
                ok = np.ones(s.n, bool)
            elif p == synth.ON:
                ok = -d[:, 2] > 0.3
            elif p == synth.ABOVE:
                ok = -d[:, 2] > 0.3
            elif p == synth.BELOW:
                ok = d[:, 2] > 0.3
            elif p in (synth.LEFT_OF, synth.RIGHT_OF):
                lat = -(d[:, :2] @ r)
                ok = (lat if p == synth.RIGHT_OF else -lat) > 0.3
            else:
                far = d[:, :2] @ fwd
                ok = (far if p == synth.IN_FRONT_OF else -far) > 0.3
            ok[o] = False
            # the anchor embedding is a noisy copy of some valid object's centroid
            cs = s.centroids.astype(np.float64) @ qb.rel_anchor[j].astype(np.float64)
            k = int(np.argmax(cs))
            assert ok[s.cls == k].any(), (qi, j, p)


def test_degenerate_scenes():
    cfg = synth.TINY
    one = synth.make_scene(cfg, n=1)
    qb = synth.make_queries(cfg, one, q=4)
    assert qb.q == 4 and (qb.planted == 0).all()
    empty = synth.make_scene(cfg, n=0)
    assert empty.desc.shape == (0, cfg.d) and empty.ids.shape == (0,)
