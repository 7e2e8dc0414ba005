"""Near over entity Gaussians (Hellinger) and the stored-view LeftOf / RightOf /
InFrontOf / Behind on the GPU against the FP64 oracle, through the C ABI.

  * exhaustive FP32 method: the full score matrix, every relation's term and
    bound anchor (each binding attains its term) and the TopK;
  * bound-pruned and learned-proposal methods, F32 / BF16 / FP8 similarity
    GEMMs: certified, the oracle's TopK; PROPOSAL equals BOUNDED bit for bit;
  * degenerate scenes (1-3 objects), anchors outside every view;
  * farm_set_entity_geometry's checks: a query naming these predicates on a
    memory without the geometry is refused (UNSUPPORTED), invalid covariances
    or views are refused (INVALID_ARG) and leave the memory unchanged.
"""
import numpy as np
import pytest

import oracle
import synth
from synth import CONFIGS, QueryBatch, make_queries, make_scene
from tests._parity import ABS, REL, assert_values_close
from tests.test_gpu_parity import _check_full, _check_topk_rows, _topk_against_full, _ws

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def farm():
    import paper_2606_15476_amd as farm
    return farm


def _geo_world(seed, n=600, q=24):
    """A mid-config scene with Gaussians and stored views; queries drawing from
    the geometry predicates and the pairwise ones; every third query has no class."""
    cfg = CONFIGS["mid"]
    scene = synth.add_entity_geometry(make_scene(cfg, n=n, seed=seed), seed)
    pool = synth.GEOMETRY_PREDS * 3 + synth.DEFAULT_PREDS + (synth.INSIDE,)
    qb = make_queries(cfg, scene, seed=seed + 1, q=q, r_min=1, r_max=4, preds=pool)
    qb.target_cls[::3] = -1
    for p in synth.GEOMETRY_PREDS:
        assert (qb.rel_pred == p).sum() >= 2, p
    return cfg, scene, qb


def test_geometry_full_parity(farm):
    cfg, scene, qb = _geo_world(51)
    mem, ws, full = _check_full(farm, scene, qb, "geometry")
    _topk_against_full(farm, mem, ws, scene, qb, full, cfg.k, "geometry")


@pytest.mark.parametrize("dtype", [0, 1, 2], ids=["f32", "bf16", "fp8"])
def test_geometry_bounded_and_proposal(farm, dtype):
    from tests import _gpu
    cfg, scene, qb = _geo_world(53)
    mem = _gpu.build_memory(scene, flags=farm.FARM_BUILD_BF16 | farm.FARM_BUILD_FP8)
    ws = _ws(farm, mem, qb)
    s64 = oracle.score(scene, qb)
    full = (s64, s64, s64)
    bd = _gpu.query_topk(mem, ws, qb, cfg.k, dtype=dtype, with_cert=True, method=farm.BOUNDED)
    assert np.all(bd[4] == 1)
    _check_topk_rows(scene, bd[0], bd[1], full, cfg.k)
    farm.build_proposals(mem, farm.ProposalNet(scene.d, max_batch=4096, seed=3), 32)
    pr = _gpu.query_topk(mem, ws, qb, cfg.k, dtype=dtype, with_cert=True, method=farm.PROPOSAL)
    for a, b in zip(pr, bd):
        np.testing.assert_array_equal(a, b)
    if dtype == 0:
        ex = _gpu.query_topk(mem, ws, qb, cfg.k, dtype=0, with_cert=True, method=farm.EXHAUSTIVE)
        for a, b in zip(bd[:4], ex[:4]):
            np.testing.assert_array_equal(a, b)
    # the breakdown of every returned object: terms and bindings against the oracle
    idx_of = {int(v): i for i, v in enumerate(scene.ids)}
    for qq in range(qb.q):
        r0, r1 = int(qb.rel_off[qq]), int(qb.rel_off[qq + 1])
        for rank in range(cfg.k):
            o = idx_of[int(bd[0][qq, rank])]
            for e in range(r1 - r0):
                j = idx_of[int(bd[3][qq, rank, e])]
                v = oracle.binding_value(scene, int(qb.rel_pred[r0 + e]), qb.rel_anchor[r0 + e], o, j,
                                         int(qb.target_cls[qq]))
                assert abs(v - bd[2][qq, rank, e]) <= REL * v + ABS, (qq, rank, e)


def test_geometry_degenerate_scenes(farm):
    """One to three objects; a scene whose views see no other object (every
    view term 0, no binding)."""
    cfg = CONFIGS["tiny"]
    rng = np.random.default_rng(9)
    for n in (1, 2, 3):
        scene = synth.add_entity_geometry(make_scene(cfg, n=n, seed=60 + n), n)
        preds = np.array([14, 15, 16, 17, 18, 14], np.int32)
        qb = QueryBatch(target=rng.standard_normal((2, cfg.d)).astype(np.float32),
                        target_cls=np.array([-1, 0], np.int32), rel_off=np.array([0, 3, 6], np.int32),
                        rel_pred=preds, rel_anchor=rng.standard_normal((6, cfg.d)).astype(np.float32),
                        planted=np.zeros(2, np.int64))
        mem, ws, full = _check_full(farm, scene, qb, f"geometry n={n}")
        _topk_against_full(farm, mem, ws, scene, qb, full, 4, f"geometry n={n}")
    # cameras looking away from the scene: every view term is 0
    scene = synth.add_entity_geometry(make_scene(cfg, n=40, seed=70), 70)
    scene.view[:, 9:12] *= -1.0   # forward reversed ...
    scene.view[:, 3:6] *= -1.0    # ... and right with it (still a rotation)
    qb = make_queries(cfg, scene, seed=71, q=6, r_min=1, r_max=2, preds=synth.VIEW_PREDS)
    _, _, t64, _ = oracle.score(scene, qb, terms=True)
    assert np.all(t64 == 0.0)
    _check_full(farm, scene, qb, "views looking away")


def test_geometry_checks(farm):
    import torch
    from tests import _gpu
    cfg = CONFIGS["tiny"]
    scene = synth.add_entity_geometry(make_scene(cfg, n=30, seed=80), 80)
    bare = synth.Scene(scene.desc, scene.center, scene.extent, scene.ids, scene.cls, scene.view_right,
                       scene.centroids)
    qb = make_queries(cfg, scene, seed=81, q=3, r_min=1, r_max=1, preds=(synth.NEAR_H,))
    qv = make_queries(cfg, scene, seed=82, q=3, r_min=1, r_max=1, preds=(synth.LEFT_OF_V,))
    mem = _gpu.build_memory(bare)
    ws = _ws(farm, mem, qb)
    out = torch.empty((3, scene.n), dtype=torch.float32, device="cuda")
    for batch in (qb, qv):
        target, anchors = _gpu.query_tensors(batch)
        with pytest.raises(farm.FarmError) as e:
            farm.score_query(mem, ws, target, batch.target_cls, batch.rel_off, batch.rel_pred, anchors, out)
        assert e.value.status == -4
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    # Gaussians only: Hellinger Near works, the view predicates are still refused
    mem.set_entity_geometry(dev(scene.cov), None)
    s, _, _ = _gpu.score_full(mem, ws, qb)
    assert_values_close(s, oracle.score(scene, qb), "Hellinger Near after attaching Gaussians")
    target, anchors = _gpu.query_tensors(qv)
    with pytest.raises(farm.FarmError) as e:
        farm.score_query(mem, ws, target, qv.target_cls, qv.rel_off, qv.rel_pred, anchors, out)
    assert e.value.status == -4
    mem.set_entity_geometry(None, dev(scene.view))
    s, _, _ = _gpu.score_full(mem, ws, qv)
    assert_values_close(s, oracle.score(scene, qv), "stored views after attaching them")
    # invalid inputs are refused and change nothing
    bad_cov = scene.cov.copy()
    bad_cov[7] = [1.0, 2.0, 0.0, 1.0, 0.0, 1.0]      # not positive definite
    bad_view = scene.view.copy()
    bad_view[4, 3:6] *= 2.0                           # rotation row not unit length
    nan_cov = scene.cov.copy()
    nan_cov[2, 0] = np.nan
    for c, v in ((bad_cov, None), (None, bad_view), (nan_cov, None)):
        with pytest.raises(farm.FarmError) as e:
            mem.set_entity_geometry(None if c is None else dev(c), None if v is None else dev(v))
        assert e.value.status == -1
    s, _, _ = _gpu.score_full(mem, ws, qb)
    assert_values_close(s, oracle.score(scene, qb), "Hellinger Near after refused updates")
    # replacing the views with other valid ones takes effect
    other = synth.add_entity_geometry(scene, 99)
    mem.set_entity_geometry(None, dev(other.view))
    s, _, _ = _gpu.score_full(mem, ws, qv)
    assert_values_close(s, oracle.score(other, qv), "replaced views")
