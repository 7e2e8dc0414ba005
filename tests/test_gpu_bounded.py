"""Exact bound-pruned TopK (FARM_METHOD_BOUNDED).

The blend keeps each score in [(1-w) s_sem, s_sem]; objects whose s_sem upper
bound falls below the K-th largest lower bound cannot enter the TopK.  Checks:
  * FP32: identical ids and bit-identical scores, terms and bound anchors to the
    exhaustive FP32 path (same similarities, same per-pair arithmetic) for all
    4,096 queries at N = 20,000, and the oracle's exact TopK on samples;
  * BF16 / FP8 similarities: every query certified, and the oracle's exact TopK.
"""
import numpy as np
import pytest

import oracle
from synth import CONFIGS, make_queries, make_scene
from tests._parity import assert_topk_valid
from tests.test_gpu_precision import _check_rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def farm():
    import paper_2606_15476_amd as farm
    return farm


@pytest.fixture(scope="module")
def world(farm):
    from tests import _gpu
    cfg = CONFIGS["precision"]
    scene = make_scene(cfg)
    qb = make_queries(cfg, scene)
    mem = _gpu.build_memory(scene, flags=farm.FARM_BUILD_BF16 | farm.FARM_BUILD_FP8)
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 64)
    return cfg, scene, qb, mem, ws


def test_bounded_f32_equals_exhaustive_full_size(farm, world):
    from tests import _gpu
    cfg, scene, qb, mem, ws = world
    ex = _gpu.query_topk(mem, ws, qb, cfg.k, with_cert=True)
    bd = _gpu.query_topk(mem, ws, qb, cfg.k, with_cert=True, method=farm.BOUNDED)
    print(f"[bounded f32] certified {int((bd[4] == 1).sum())}/{qb.q}", flush=True)
    assert np.all(bd[4] == 1)
    np.testing.assert_array_equal(bd[0], ex[0])
    np.testing.assert_array_equal(bd[1], ex[1])
    np.testing.assert_array_equal(bd[2], ex[2])
    np.testing.assert_array_equal(bd[3], ex[3])


@pytest.mark.parametrize("dtype", [1, 2], ids=["bf16", "fp8"])
def test_bounded_reduced_precision_is_exact(farm, world, dtype):
    from tests import _gpu
    cfg, scene, qb, mem, ws = world
    ids, sc, terms, anch, cert = _gpu.query_topk(mem, ws, qb, cfg.k, dtype=dtype, with_cert=True,
                                                 method=farm.BOUNDED)
    ex = _gpu.query_topk(mem, ws, qb, cfg.k)
    print(f"[bounded dtype={dtype}] certified {int((cert == 1).sum())}/{qb.q}", flush=True)
    assert np.all(cert == 1)
    # same ids as the exact path wherever the exact scores are separated by more than the FP32 tolerance
    gaps_ok = 0
    for qq in range(qb.q):
        if list(ids[qq]) != list(ex[0][qq]):
            d = np.abs(sc[qq] - ex[1][qq])
            # both within 1e-5 * max(s, 0.01) of the oracle's scores
            assert np.all(d <= 2e-5 * np.maximum(np.abs(ex[1][qq]), 1e-2)), qq
        else:
            gaps_ok += 1
    rows = list(np.random.default_rng(5).choice(qb.q, size=12, replace=False))
    oidx, osc, ot, ob, ns = oracle.topk_bounded(scene, qb.subset(rows), cfg.k + 6)
    _check_rows(scene, qb, rows, ids, sc, terms, anch, cert, oidx, osc, cfg.k)


def test_bounded_small_and_ragged(farm):
    from tests import _gpu
    from tests.test_gpu_parity import _random_queries, _random_scene
    for n, d in ((1, 8), (7, 16), (600, 40)):
        scene = _random_scene(n, d, seed=n)
        qb = _random_queries(scene, 5, [0, 2, 3], seed=n + 1)
        mem = _gpu.build_memory(scene, flags=farm.FARM_BUILD_BF16 | farm.FARM_BUILD_FP8)
        ws = farm.Workspace(mem, qb.q, qb.r_tot, 64)
        s64 = oracle.score(scene, qb)
        for dt in (0, 1, 2):
            ids, sc, terms, anch, cert = _gpu.query_topk(mem, ws, qb, 10, dtype=dt, with_cert=True,
                                                         method=farm.BOUNDED)
            assert np.all(cert == 1)
            for qq in range(qb.q):
                order = oracle.topk(s64[qq], scene.ids, min(n, 18))
                by_id = {int(v): s64[qq, i] for i, v in enumerate(scene.ids)}
                assert_topk_valid(ids[qq], sc[qq], scene.ids[order], s64[qq, order], lambda g: by_id[g], 10)


@pytest.mark.parametrize("k", [1, 16, 17, 64, 300])
def test_bounded_and_proposal_k_range(farm, k):
    """Both K forms of the candidate scan (per-thread top-16 lists for K <= 16, radix select above) against
    the exhaustive FP32 path: same ids and bit-identical scores for FP32 similarities."""
    from tests import _gpu
    cfg = CONFIGS["mid"]
    scene = make_scene(cfg, n=1500, seed=21)
    qb = make_queries(cfg, scene, seed=22, q=48)
    mem = _gpu.build_memory(scene, flags=farm.FARM_BUILD_BF16)
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 512)
    ex = _gpu.query_topk(mem, ws, qb, k)
    bd = _gpu.query_topk(mem, ws, qb, k, with_cert=True, method=farm.BOUNDED)
    assert np.all(bd[4] == 1)
    np.testing.assert_array_equal(bd[0], ex[0])
    np.testing.assert_array_equal(bd[1], ex[1])
    net = farm.ProposalNet(scene.d, max_batch=256, seed=4)
    farm.build_proposals(mem, net, 64)
    pr = _gpu.query_topk(mem, ws, qb, k, with_cert=True, method=farm.PROPOSAL)
    for a, b in zip(pr, bd):
        np.testing.assert_array_equal(a, b)


def test_bounded_candidate_overflow_is_reported(farm):
    """More than 2,048 objects that can reach the TopK (identical descriptors): the query is reported
    uncertified, and the answer is still a valid ranking of scored objects."""
    from tests import _gpu
    from tests.test_gpu_parity import _random_queries, _random_scene
    scene = _random_scene(3000, 32, seed=8)
    scene.desc[:] = scene.desc[0]
    if scene.cls is not None:
        scene.cls[:] = -1  # no class factor: every object has the same s_sem
    qb = _random_queries(scene, 4, [0, 1, 2], seed=9)
    mem = _gpu.build_memory(scene)
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 16)
    ids, sc, terms, anch, cert = _gpu.query_topk(mem, ws, qb, 10, with_cert=True, method=farm.BOUNDED)
    assert np.all(cert == 0)
    s_full = _gpu.score_full(mem, ws, qb, terms=False)
    idx_of = {int(v): i for i, v in enumerate(scene.ids)}
    for qq in range(qb.q):
        assert np.all(np.diff(sc[qq]) <= 0)
        for rank in range(10):
            i = idx_of[int(ids[qq, rank])]
            assert sc[qq, rank] == s_full[qq, i]  # each returned score is that object's exact score
