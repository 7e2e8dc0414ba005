"""Pins of the multi-channel reciprocal-rank fusion oracle (oracle/rrf.py) and of the
oracle's scoring with supplied unary scores (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from oracle import rrf
from oracle.brute import brute_scores
from synth import QueryBatch, Scene

MU = 5.0


def _angles_space(angles_deg):
    a = np.radians(np.asarray(angles_deg, np.float64))
    return np.stack([np.cos(a), np.sin(a)], axis=1)


def test_worked_example_two_channels():
    """Four entities; channel 0 (weight 1.0) sees them at 10, 40, 70, 100 degrees from its query
    (ranks 1, 2, 3, 4), channel 1 (weight 0.5, another space) at 80, 5, 60, 20 degrees (ranks 4, 1,
    3, 2).  Fused score = (1/(5 + r0) + 0.5/(5 + r1)) / (1.5/6)."""
    ids = np.array([7, 3, 9, 1], np.uint32)
    s0 = _angles_space([10, 40, 70, 100])
    s1 = _angles_space([80, 5, 60, 20])
    q = np.array([[1.0, 0.0]])
    got = rrf.fused([s0, s1], ids, [(0, 1.0, q), (1, 0.5, q)], "target")[0]
    r0, r1 = [1, 2, 3, 4], [4, 1, 3, 2]
    want = [(1.0 / (MU + a) + 0.5 / (MU + b)) / (1.5 / (MU + 1.0)) for a, b in zip(r0, r1)]
    np.testing.assert_allclose(got, want, rtol=1e-15)
    assert got[0] == pytest.approx((1 / 6 + 0.5 / 9) * 4, rel=1e-15)


def test_equal_cosines_rank_by_id_and_ranks_are_a_permutation():
    rng = np.random.default_rng(1)
    n = 40
    ids = rng.permutation(1000)[:n].astype(np.uint32)
    cos = np.round(rng.uniform(-1, 1, (5, n)), 1)   # many exact ties
    rk = rrf.channel_ranks(cos, ids)
    for r in range(5):
        assert sorted(rk[r]) == list(range(1, n + 1))
        for i in range(n):   # brute force: 1 + the number of entities before i
            before = sum(1 for j in range(n) if cos[r, j] > cos[r, i] or (cos[r, j] == cos[r, i] and ids[j] < ids[i]))
            assert rk[r, i] == 1 + before


def test_tolerant_ranks_bracket_the_exact_one():
    rng = np.random.default_rng(2)
    n = 200
    ids = rng.permutation(10 ** 6)[:n].astype(np.uint32)
    cos = rng.normal(0, 0.03, (3, n))
    cos[:, 5] = cos[:, 6] + 1e-7   # near ties
    ex = rrf.channel_ranks(cos, ids)
    lo = rrf.channel_ranks(cos, ids, -1, 1e-6)
    hi = rrf.channel_ranks(cos, ids, +1, 1e-6)
    assert np.all(lo <= ex) and np.all(ex <= hi)
    assert np.any(hi > lo)
    # eps = 0: the bounds differ from the exact rank only through equal cosines (none here)
    np.testing.assert_array_equal(rrf.channel_ranks(cos, ids, -1, 0.0), ex)
    np.testing.assert_array_equal(rrf.channel_ranks(cos, ids, +1, 0.0), ex)


def test_channel_weights_add_and_single_channel_keeps_the_cosine_order():
    rng = np.random.default_rng(3)
    n = 60
    ids = np.arange(1, n + 1, dtype=np.uint32)
    sp = [rng.standard_normal((n, 8)), rng.standard_normal((n, 5))]
    qa, qb_ = rng.standard_normal((2, 8)), rng.standard_normal((2, 5))
    a = rrf.fused(sp, ids, [(0, 0.25, qa), (0, 0.5, qa), (1, 1.0, qb_)], "target")
    b = rrf.fused(sp, ids, [(0, 0.75, qa), (1, 1.0, qb_)], "target")
    np.testing.assert_allclose(a, b, rtol=1e-14)
    one = rrf.fused(sp, ids, [(1, 2.0, qb_)], "target")
    cos = (qb_ / np.linalg.norm(qb_, axis=1, keepdims=True)) @ (sp[1] / np.linalg.norm(sp[1], axis=1, keepdims=True)).T
    for r in range(2):
        assert np.all(np.diff(one[r][np.argsort(-cos[r], kind="stable")]) <= 0)
        assert one[r].max() == pytest.approx(1.0) and one[r].min() > 0


def _tiny_scene(seed, n, r, q=3, d=6):
    rng = np.random.default_rng(seed)
    cls = rng.integers(0, 3, n).astype(np.int32)
    scene = Scene(desc=rng.standard_normal((n, d)).astype(np.float32),
                  center=rng.uniform(0, 2, (n, 3)).astype(np.float32),
                  extent=rng.uniform(0.2, 1.5, (n, 3)).astype(np.float32),
                  ids=(rng.permutation(100)[:n] + 1).astype(np.uint32), cls=cls,
                  view_right=np.array([math.cos(seed), math.sin(seed)], np.float32),
                  centroids=np.zeros((3, d), np.float32))
    preds = rng.integers(0, 9, q * r).astype(np.int32)
    qb = QueryBatch(target=rng.standard_normal((q, d)).astype(np.float32),
                    target_cls=rng.integers(-1, 3, q).astype(np.int32),
                    rel_off=np.arange(0, q * r + 1, r, dtype=np.int32), rel_pred=preds,
                    rel_anchor=rng.standard_normal((q * r, d)).astype(np.float32), planted=np.zeros(q, np.int64))
    return scene, qb


def test_supplied_unary_scores_reproduce_the_cosine_path():
    """Handing the oracle the clamped cosines it would compute itself changes nothing (every query
    reads its own rows, relations at their CSR offsets)."""
    scene, qb = _tiny_scene(4, 30, 3, q=5)
    u = scene.desc.astype(np.float64)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    unit = lambda v: np.asarray(v, np.float64) / np.linalg.norm(np.asarray(v, np.float64), axis=1, keepdims=True)
    sem = np.maximum(0, unit(qb.target) @ u.T)
    kappa = np.where((qb.target_cls[:, None] >= 0) & (scene.cls[None, :] != qb.target_cls[:, None]), 0.3, 1.0)
    asim = np.maximum(0, unit(qb.rel_anchor) @ u.T)
    ref, rsem, rt, rb = oracle.score(scene, qb, terms=True)
    with oracle.similarities(sem * kappa, asim):
        got, gsem, gt, gb = oracle.score(scene, qb, terms=True)
    np.testing.assert_allclose(got, ref, rtol=1e-12)
    np.testing.assert_allclose(gt, rt, rtol=1e-12)
    np.testing.assert_array_equal(gb, rb)


@pytest.mark.parametrize("n,r", [(2, 1), (5, 2), (7, 3)])
def test_fused_scores_star_decomposition_equals_joint_enumeration(n, r):
    """Scores with the fused unary scores: the oracle's star decomposition against the joint
    enumeration over every binding, both given the same unary rows."""
    for seed in range(3):
        scene, qb = _tiny_scene(seed * 7 + n + r, n, r)
        rng = np.random.default_rng(seed)
        spaces = [scene.desc.astype(np.float64), rng.standard_normal((n, 4))]
        tch = [(0, 1.0, qb.target), (1, 0.75, rng.standard_normal((qb.q, 4)))]
        ach = [(0, 1.0, qb.rel_anchor), (1, 0.75, rng.standard_normal((qb.r_tot, 4)))]
        sem, asim = rrf.similarities(scene, spaces, tch, ach, qb.target_cls)
        with oracle.similarities(sem, asim):
            s = oracle.score(scene, qb)
        bs = np.asarray(brute_scores(scene, qb, sims=(sem, asim)))
        np.testing.assert_allclose(s, bs, rtol=1e-12, atol=1e-14)
