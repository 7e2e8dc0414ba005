"""Request loop over resident scenes (farm_server_*).

  * a request's answer is the same alone and in a mixed, continuously batched
    stream of requests over several scenes of different sizes, and equals the
    direct farm_query_topk answer of the same query;
  * a budget that holds one workspace at a time defers batches (and releases
    idle workspaces) instead of failing, with the same answers;
  * a budget below any workspace leaves requests pending, without errors;
  * cancelled requests complete as cancelled and do not disturb the others;
  * requests over all twelve predicates batch like the others.
"""
import time

import numpy as np
import pytest

from synth import CONFIGS, make_queries, make_scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def farm():
    import paper_2606_15476_amd as farm
    return farm


@pytest.fixture(scope="module")
def scenes(farm):
    from tests import _gpu
    cfg = CONFIGS["precision"]
    out = []
    for i, n in enumerate((300, 1500, 4000)):
        sc = make_scene(cfg, seed=3000 + i, n=n)
        qb = make_queries(cfg, sc, seed=3100 + i, q=24)
        mem = _gpu.build_memory(sc, flags=farm.FARM_BUILD_BF16)
        out.append((sc, qb, mem))
    return out


def _requests(scenes):
    reqs = []
    for s, (sc, qb, mem) in enumerate(scenes):
        d = sc.d
        for qi in range(qb.q):
            r0, r1 = qb.rel_off[qi], qb.rel_off[qi + 1]
            reqs.append((s, qb.target[qi], int(qb.target_cls[qi]), qb.rel_pred[r0:r1],
                         qb.rel_anchor.reshape(-1, d)[r0:r1]))
    order = np.random.default_rng(0).permutation(len(reqs))
    return [reqs[i] for i in order]


def _run(farm, scenes, reqs, cancel=(), timeout=60.0, **cfg):
    sv = farm.Server(**cfg)
    for sc, qb, mem in scenes:
        sv.add_scene(mem)
    ids = [sv.submit(*r) for r in reqs]
    for i in cancel:
        sv.cancel(ids[i])
    res = {}
    t0 = time.time()
    while len(res) < len(ids):
        sv.progress()
        for rid, st, ce, lat, tid, tsc in sv.poll():
            res[rid] = (st, ce, tid, tsc)
        assert time.time() - t0 < timeout, "serving loop did not finish"
    stats = sv.stats()
    sv.close()
    return [res[i] for i in ids], stats


@pytest.mark.parametrize("dtype,method", [(0, 0), (1, 1), (1, 2)], ids=["f32-exhaustive", "bf16-bounded",
                                                                         "bf16-proposal"])
def test_alone_equals_mix(farm, scenes, dtype, method):
    if method == farm.PROPOSAL:
        net = farm.ProposalNet(scenes[0][0].d, max_batch=256, seed=3)
        for _, _, mem in scenes:
            farm.build_proposals(mem, net, 64)
    reqs = _requests(scenes)
    alone = []
    for r in reqs:
        out, _ = _run(farm, scenes, [r], slots=1, max_batch_q=1, max_batch_rel=8, dtype=dtype, method=method)
        alone.append(out[0])
    mix, stats = _run(farm, scenes, reqs, slots=3, max_batch_q=16, max_batch_rel=64, dtype=dtype, method=method)
    print(f"[serve] {stats}", flush=True)
    assert stats["batches"] < len(reqs)  # requests were batched together
    for a, m in zip(alone, mix):
        assert a[0] == 0 and m[0] == 0
        np.testing.assert_array_equal(a[2], m[2])
        np.testing.assert_array_equal(a[3], m[3])
    # and equal to the direct call of the library on the same queries
    from tests import _gpu
    for s, (sc, qb, mem) in enumerate(scenes):
        ws = farm.Workspace(mem, qb.q, qb.r_tot, 16)
        ids, sco = _gpu.query_topk(mem, ws, qb, 10, dtype=dtype, method=method)[:2]
        for (rs, tgt, *_), m in zip(reqs, mix):
            if rs != s:
                continue
            qi = int(np.where((qb.target == tgt).all(axis=1))[0][0])
            np.testing.assert_array_equal(m[2], ids[qi])
            np.testing.assert_array_equal(m[3], sco[qi])


def test_tight_budget_defers(farm, scenes):
    import paper_2606_15476_amd as f
    reqs = _requests(scenes)
    largest = max(f.workspace_estimate(mem, 16, 64, 10) for _, _, mem in scenes)
    ref, _ = _run(farm, scenes, reqs, slots=3, max_batch_q=16, max_batch_rel=64)
    tight, stats = _run(farm, scenes, reqs, slots=3, max_batch_q=16, max_batch_rel=64, hbm_budget=largest)
    print(f"[serve tight] {stats}", flush=True)
    assert stats["deferrals"] > 0 and stats["evictions"] > 0
    assert stats["bytes_held"] <= largest
    for a, b in zip(ref, tight):
        assert b[0] == 0
        np.testing.assert_array_equal(a[2], b[2])
        np.testing.assert_array_equal(a[3], b[3])


def test_budget_below_any_workspace_keeps_pending(farm, scenes):
    sv = farm.Server(slots=2, max_batch_q=8, max_batch_rel=32, hbm_budget=1024)
    for _, _, mem in scenes:
        sv.add_scene(mem)
    for r in _requests(scenes)[:5]:
        sv.submit(*r)
    for _ in range(20):
        busy, pending = sv.progress()
        assert busy == 0 and pending == 5
    assert sv.poll() == []
    assert sv.stats()["deferrals"] >= 20
    sv.close()


def test_cancel_leaves_others_intact(farm, scenes):
    reqs = _requests(scenes)
    ref, _ = _run(farm, scenes, reqs, slots=2, max_batch_q=8, max_batch_rel=32)
    cancel = (0, 5, 17, len(reqs) - 1)
    got, _ = _run(farm, scenes, reqs, cancel=cancel, slots=2, max_batch_q=8, max_batch_rel=32)
    for i, (a, b) in enumerate(zip(ref, got)):
        if i in cancel:
            assert b[0] == 1
        else:
            assert b[0] == 0
            np.testing.assert_array_equal(a[2], b[2])
            np.testing.assert_array_equal(a[3], b[3])


def test_invalid_requests_rejected(farm, scenes):
    sv = farm.Server(slots=1, max_batch_q=4, max_batch_rel=8)
    sc, qb, mem = scenes[0]
    sv.add_scene(mem)
    d = sc.d
    good_t = qb.target[0]
    bad = [
        (0, np.zeros(d, np.float32), -1, [0], np.ones((1, d), np.float32)),          # zero target
        (0, np.full(d, np.nan, np.float32), -1, [0], np.ones((1, d), np.float32)),   # NaN target
        (0, good_t, -1, [farm.NUM_PRED], np.ones((1, d), np.float32)),               # bad predicate
        (0, good_t, -1, [0] * 9, np.ones((9, d), np.float32)),                       # R > 8
        (5, good_t, -1, [0], np.ones((1, d), np.float32)),                           # unknown scene
        (0, good_t[: d - 1], -1, [0], np.ones((1, d - 1), np.float32)),              # width
    ]
    for r in bad:
        with pytest.raises(farm.FarmError):
            sv.submit(*r)
    assert sv.progress() == (0, 0)
    sv.close()


def test_every_predicate_mix_equals_direct(farm):
    """Requests drawing from all twelve predicates (On, Closest, Farthest and
    Inside included), batched across scenes: the same answers as the direct
    library call on the same queries (BF16 learned-proposal form)."""
    import synth
    from tests import _gpu
    cfg = CONFIGS["precision"]
    scenes = []
    for i, n in enumerate((400, 1200)):
        sc = make_scene(cfg, seed=3200 + i, n=n)
        qb = make_queries(cfg, sc, seed=3300 + i, q=20, preds=synth.EVERY_PRED)
        mem = _gpu.build_memory(sc, flags=farm.FARM_BUILD_BF16)
        scenes.append((sc, qb, mem))
    net = farm.ProposalNet(scenes[0][0].d, max_batch=256, seed=4)
    for _, _, mem in scenes:
        farm.build_proposals(mem, net, 64)
    reqs = _requests(scenes)
    mix, stats = _run(farm, scenes, reqs, slots=2, max_batch_q=8, max_batch_rel=32, dtype=1, method=farm.PROPOSAL)
    assert stats["batches"] < len(reqs)
    for s, (sc, qb, mem) in enumerate(scenes):
        ws = farm.Workspace(mem, qb.q, qb.r_tot, 16)
        ids, sco = _gpu.query_topk(mem, ws, qb, 10, dtype=1, method=farm.PROPOSAL)[:2]
        for (rs, tgt, *_), m in zip(reqs, mix):
            if rs != s:
                continue
            assert m[0] == 0
            qi = int(np.where((qb.target == tgt).all(axis=1))[0][0])
            np.testing.assert_array_equal(m[2], ids[qi])
            np.testing.assert_array_equal(m[3], sco[qi])
