"""Learned anchor proposals (farm_build_proposals, FARM_METHOD_PROPOSAL).

  * tables: every list holds M distinct anchors other than its target, the
    cached predicate values equal the oracle's P_p(o, a), the stored bound is the
    oracle's largest P_p(o, a) over the anchors left out, and a list is the top
    M of the network's own logits;
  * exactness: the proposal method returns the same ids, scores, terms and bound
    anchors as the bound-pruned method (which is the exact TopK, tested against
    the exhaustive path and the oracle elsewhere) for FP32, BF16 and FP8
    similarities, with any network -- trained or not -- since uncertified terms
    fall back to the scan over all anchors;
  * gain: on a held-out scene of the same generator, a network trained on the
    exhaustive pass's bindings certifies more terms than an untrained one and
    beats the method without lists; lists ranked by the exact predicate value
    (the non-learned baseline) are measured beside it;
  * the default benchmark form at full size: 256 fixed queries of the
    4,096-query launch against the oracle's exact TopK.
"""
import numpy as np
import pytest

import oracle
from synth import CONFIGS, make_queries, make_scene

pytestmark = pytest.mark.gpu

REL, ABS = 1e-5, 4e-6


@pytest.fixture(scope="module")
def farm():
    import paper_2606_15476_amd as farm
    return farm


def _tables(farm, mem):
    m, idx, val, out = farm.get_proposals(mem)
    return m, idx.cpu().numpy(), val.cpu().numpy(), out.cpu().numpy()


def _p64(scene, p, o, a):
    return oracle.predicate(p, scene.center[o], scene.center[a], scene.view_right, scene.extent[o], scene.extent[a])


def test_tables_match_oracle(farm):
    import torch
    from tests import _gpu
    scene = make_scene(CONFIGS["mid"], n=600, seed=11)
    mem = _gpu.build_memory(scene)
    net = farm.ProposalNet(scene.d, max_batch=4096, seed=5)
    farm.build_proposals(mem, net, 48)
    m, idx, val, out = _tables(farm, mem)
    n = scene.n
    assert m == 48 and idx.shape == (farm.NUM_PROP_PRED, n, m)
    rng = np.random.default_rng(0)
    for o in rng.choice(n, 12, replace=False):
        for p in range(farm.NUM_PROP_PRED):
            lst = idx[p, o]
            assert np.all((lst >= 0) & (lst < n)) and np.all(lst != o)
            assert len(set(lst.tolist())) == m
            # cached values: log P for the Gaussians (Near, NextTo, On), P otherwise
            log_domain = p in (farm.NEAR, farm.NEXT_TO, farm.ON)
            for e, a in enumerate(lst):
                v64 = _p64(scene, p, o, a)
                got = np.exp(np.float64(val[p, o, e])) if log_domain else np.float64(val[p, o, e])
                assert abs(got - v64) <= REL * abs(v64) + ABS, (o, p, a, got, v64)
            # bound over the anchors left out
            rest = [a for a in range(n) if a != o and a not in set(lst.tolist())]
            pout64 = max(_p64(scene, p, o, a) for a in rest)
            got = np.exp(np.float64(out[p, o])) if log_domain else np.float64(out[p, o])
            assert abs(got - pout64) <= REL * abs(pout64) + ABS, (o, p, got, pout64)
        # the lists are the network's top M (up to logit rounding of the factorised first layer)
        o_t = torch.full((n,), int(o), dtype=torch.int32, device="cuda")
        a_t = torch.arange(n, dtype=torch.int32, device="cuda")
        lg = torch.empty((n, farm.NUM_PROP_PRED), dtype=torch.float32, device="cuda")
        net.logits(mem, o_t, a_t, lg)
        torch.cuda.synchronize()
        lg = lg.cpu().numpy()
        lg[o] = -np.inf
        for p in range(farm.NUM_PROP_PRED):
            top = set(np.argsort(-lg[:, p], kind="stable")[:m].tolist())
            overlap = len(top & set(idx[p, o].tolist())) / m
            assert overlap >= 0.9, (o, p, overlap)


def _compare(farm, mem, ws, qb, k, dtype):
    """PROPOSAL (LDS-staged and global-memory forms of its pass) against BOUNDED."""
    from tests import _gpu
    bd = _gpu.query_topk(mem, ws, qb, k, dtype=dtype, with_cert=True, method=farm.BOUNDED)
    ws.proposal_stats(reset=True)
    pr = _gpu.query_topk(mem, ws, qb, k, dtype=dtype, with_cert=True, method=farm.PROPOSAL)
    checked, fell = ws.proposal_stats(reset=True)[:2]
    for a, b in zip(pr, bd):
        np.testing.assert_array_equal(a, b)
    pg = _gpu.query_topk(mem, ws, qb, k, dtype=dtype, with_cert=True, method=farm.PROPOSAL,
                         flags=farm.OPT_GLOBAL_PROPOSAL_PASS)
    ws.proposal_stats(reset=True)
    for a, b in zip(pg, bd):
        np.testing.assert_array_equal(a, b)
    return checked, fell


@pytest.mark.parametrize("m", [256, 300, 254], ids=["m256", "m300", "m254"])
@pytest.mark.parametrize("dtype", [0, 1, 2], ids=["f32", "bf16", "fp8"])
def test_proposal_equals_bounded_mid(farm, dtype, m):
    """Lists of at most 256 entries in multiples of 4 take the register form, others the general one."""
    from tests import _gpu
    cfg = CONFIGS["mid"]
    scene = make_scene(cfg)
    qb = make_queries(cfg, scene)
    mem = _gpu.build_memory(scene, flags=farm.FARM_BUILD_BF16 | farm.FARM_BUILD_FP8)
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 64)
    net = farm.ProposalNet(scene.d, max_batch=4096, seed=1)
    farm.build_proposals(mem, net, m)
    assert farm.get_proposals(mem)[0] == m
    checked, fell = _compare(farm, mem, ws, qb, cfg.k, dtype)
    print(f"[proposal mid dtype={dtype} m={m}] terms {checked}, fell back {fell}", flush=True)
    assert checked > 0 and 0 <= fell <= checked


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "bf16"])
def test_all_predicates(farm, dtype):
    """Lists for NextTo/InFrontOf/Behind/On too (their depth coordinates, the
    log domain of NextTo and On, On's bottom/top faces); results stay
    bit-identical to BOUNDED, which equals the exact TopK."""
    import synth
    from tests import _gpu
    cfg = CONFIGS["mid"]
    scene = make_scene(cfg, seed=23)
    qb = make_queries(cfg, scene, seed=24, q=64, preds=synth.ALL_PREDS)
    mem = _gpu.build_memory(scene, flags=farm.FARM_BUILD_BF16)
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 64)
    net = farm.ProposalNet(scene.d, max_batch=4096, seed=5)
    farm.build_proposals(mem, net, 64)
    checked, fell = _compare(farm, mem, ws, qb, cfg.k, dtype)
    # and BOUNDED (hence PROPOSAL) is the exact TopK of the oracle
    from tests.test_gpu_parity import _check_bounded
    ids, sc, _, _, cert = _gpu.query_topk(mem, ws, qb, cfg.k, dtype=dtype, with_cert=True, method=farm.BOUNDED)
    assert np.all(cert == 1)
    oidx, osc, ot, ob, ns = oracle.topk_bounded(scene, qb, cfg.k + 8)
    _check_bounded(scene, qb, ids, sc, oidx, osc, cfg.k)
    print(f"[proposal all predicates dtype={dtype}] terms {checked}, fell back {fell}", flush=True)
    assert checked > 0 and fell < checked


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "bf16"])
def test_rank_predicates(farm, dtype):
    """Closest/Farthest and Inside have no lists: every such term takes the
    full-scan fallback (LDS-staged and global-memory forms of the pass); results stay
    bit-identical to BOUNDED, which equals the exact TopK."""
    from tests import _gpu
    from tests._parity import oracle_bounds
    from tests.test_gpu_parity import _check_topk_rows, _rank_world
    cfg, scene, qb = _rank_world(35)
    mem = _gpu.build_memory(scene, flags=farm.FARM_BUILD_BF16)
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 64)
    net = farm.ProposalNet(scene.d, max_batch=4096, seed=5)
    farm.build_proposals(mem, net, 64)
    checked, fell = _compare(farm, mem, ws, qb, cfg.k, dtype)
    ids, sc, _, _, cert = _gpu.query_topk(mem, ws, qb, cfg.k, dtype=dtype, with_cert=True, method=farm.BOUNDED)
    assert np.all(cert == 1)
    s64, _, _, _, s_lo, s_hi, _, _ = oracle_bounds(scene, qb)
    _check_topk_rows(scene, ids, sc, (s64, s_lo, s_hi), cfg.k)
    print(f"[proposal rank predicates dtype={dtype}] terms {checked}, fell back {fell}", flush=True)
    assert checked > 0 and fell > 0


def test_proposal_equals_bounded_full_size(farm):
    from tests import _gpu
    cfg = CONFIGS["precision"]
    scene = make_scene(cfg)
    qb = make_queries(cfg, scene)
    mem = _gpu.build_memory(scene, flags=farm.FARM_BUILD_BF16)
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 64)
    net = farm.ProposalNet(scene.d, max_batch=4096, seed=2)
    farm.build_proposals(mem, net, 256)
    for dtype in (0, 1):
        checked, fell = _compare(farm, mem, ws, qb, cfg.k, dtype)
        print(f"[proposal full dtype={dtype}] terms {checked}, fell back {fell}", flush=True)
        assert checked > 0


def test_small_scenes_and_errors(farm):
    import torch
    from tests import _gpu
    from tests.test_gpu_parity import _random_queries, _random_scene
    for n, d, m in ((1, 8, 4), (2, 8, 4), (7, 16, 64), (300, 40, 32)):
        scene = _random_scene(n, d, seed=n)
        qb = _random_queries(scene, 5, [0, 2, 3], seed=n + 1)
        mem = _gpu.build_memory(scene, flags=farm.FARM_BUILD_BF16)
        ws = farm.Workspace(mem, qb.q, qb.r_tot, 16)
        with pytest.raises(farm.FarmError) if n >= 2 else _nullctx():
            _gpu.query_topk(mem, ws, qb, 10, method=farm.PROPOSAL)
        net = farm.ProposalNet(d, max_batch=256, seed=n)
        farm.build_proposals(mem, net, m)
        got_m = farm.get_proposals(mem)[0]
        assert got_m == min(m, n - 1) if n >= 2 else got_m == 0
        for dtype in (0, 1):
            _compare(farm, mem, ws, qb, 10, dtype)
    # width mismatch
    scene = _random_scene(20, 16, seed=3)
    mem = _gpu.build_memory(scene)
    net = farm.ProposalNet(32, max_batch=64, seed=0)
    with pytest.raises(farm.FarmError):
        farm.build_proposals(mem, net, 8)
    net16 = farm.ProposalNet(16, max_batch=64, seed=0)
    for bad_m in (0, farm.FARM_MAX_K + 1):
        with pytest.raises(farm.FarmError):
            farm.build_proposals(mem, net16, bad_m)


class _nullctx:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


def _timed(farm, mem, ws, qb, k, dtype, method, reps=5):
    """Median ms of one farm_query_topk batch (HIP events around the call on the current stream)."""
    import torch
    from tests import _gpu
    target, anchors = _gpu.query_tensors(qb)
    oid = torch.empty((qb.q, k), dtype=torch.int32, device="cuda")
    osc = torch.empty((qb.q, k), dtype=torch.float32, device="cuda")
    times = []
    for _ in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        farm.query_topk(mem, ws, target, qb.target_cls, qb.rel_off, qb.rel_pred, anchors, k, oid, osc, dtype=dtype,
                        method=method)
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b))
    return float(np.median(times[1:]))


def test_trained_network_gain(farm):
    """What the trained network gains, on a held-out scene of the generator:
    against the method without lists (BOUNDED: every candidate term scanned
    over all anchors), against an untrained network, and beside the
    non-learned baseline -- lists ranked by the exact predicate value P(o, a),
    which have the tightest possible bound on the anchors left out.  All four
    return the same TopK."""
    from paper_2606_15476_amd import proposal
    from tests import _gpu
    import time
    cfg = CONFIGS["precision"]
    n, q = 4000, 512
    data, keep = [], []
    for seed in (1000, 1001):
        scene = make_scene(cfg, seed=seed, n=n)
        qb = make_queries(cfg, scene, seed=seed, q=q)
        mem = _gpu.build_memory(scene)
        ws = farm.Workspace(mem, qb.q, qb.r_tot, 16)
        target, anchors = _gpu.query_tensors(qb)
        bind = proposal.exhaustive_bindings(mem, ws, target, qb.target_cls, qb.rel_off, qb.rel_pred, anchors)
        o, a, p, y = proposal.sample_pairs(bind, scene.ids, qb.rel_pred, np.random.default_rng(seed),
                                           per_relation=96, negatives=3)
        data.append((mem, o, a, p, y))
        keep.append(ws)
    net = farm.ProposalNet(data[0][0].d, max_batch=4096, seed=7)
    t0 = time.time()
    hist = proposal.train(net, data, steps=400, batch=4096, lr=2e-3, weight_decay=1e-4)
    print(f"[train] {time.time() - t0:.1f}s loss {hist[0][1]:.4f} -> {hist[-1][1]:.4f}", flush=True)
    assert hist[-1][1] < hist[0][1]
    scene = make_scene(cfg, seed=2000, n=n)
    qb = make_queries(cfg, scene, seed=2000, q=q)
    mem = _gpu.build_memory(scene, flags=farm.FARM_BUILD_BF16)
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 16)
    ms_bounded = _timed(farm, mem, ws, qb, cfg.k, 1, farm.BOUNDED)
    ws.proposal_stats(reset=True)
    _gpu.query_topk(mem, ws, qb, cfg.k, dtype=1, method=farm.BOUNDED)
    full_terms = ws.proposal_stats(reset=True)[0]
    print(f"[gain] BOUNDED (no lists): {full_terms} terms scanned over all anchors, {ms_bounded:.3f} ms", flush=True)
    res = {}
    builders = (("untrained", lambda: farm.build_proposals(mem, farm.ProposalNet(mem.d, max_batch=4096, seed=7), 256)),
                ("trained", lambda: farm.build_proposals(mem, net, 256)),
                ("by value", lambda: farm.build_proposals_by_value(mem, 256)))
    for name, build in builders:
        build()
        checked, fell = _compare(farm, mem, ws, qb, cfg.k, 1)
        ms = _timed(farm, mem, ws, qb, cfg.k, 1, farm.PROPOSAL)
        res[name] = (fell / max(checked, 1), ms)
        print(f"[gain] {name}: terms {checked}, fell back {fell} ({res[name][0]:.4f}), {ms:.3f} ms", flush=True)
        assert checked == full_terms
    assert res["trained"][0] < res["untrained"][0]
    assert res["trained"][0] < 0.25 and res["trained"][1] < ms_bounded
    # the value-ranked lists are the query-independent optimum of the bound on
    # left-out anchors; the trained network comes within a small factor of it
    assert res["by value"][1] < ms_bounded
    assert res["trained"][0] <= 2.5 * res["by value"][0]


@pytest.mark.parametrize("dtype", [0, 1], ids=["f32", "bf16"])
def test_lists_by_value(farm, dtype):
    """The non-learned lists: each holds the M anchors of largest exact
    predicate value, Pout is the largest value left out, and PROPOSAL with them
    returns BOUNDED's records bit for bit."""
    from tests import _gpu
    cfg = CONFIGS["mid"]
    scene = make_scene(cfg, n=500, seed=71)
    qb = make_queries(cfg, scene, seed=72, q=48)
    mem = _gpu.build_memory(scene, flags=farm.FARM_BUILD_BF16)
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 64)
    M = 24
    farm.build_proposals_by_value(mem, M)
    m, idx, val, out = _tables(farm, mem)
    assert m == M
    rng = np.random.default_rng(1)
    for o in rng.choice(scene.n, 6, replace=False):
        for p in range(farm.NUM_PROP_PRED):
            log_domain = p in (farm.NEAR, farm.NEXT_TO, farm.ON)
            v = np.array([_p64(scene, p, o, a) for a in range(scene.n)])
            v[o] = -np.inf
            lst = idx[p, o]
            assert len(set(lst.tolist())) == M and o not in lst
            rest = np.setdiff1d(np.arange(scene.n), np.append(lst, o))
            # every listed anchor's value reaches every left-out one's (FP32 evaluation: 1e-5 slack)
            assert v[lst].min() >= v[rest].max() * (1 - 1e-5) - 4e-6, (o, p)
            got_out = np.exp(np.float64(out[p, o])) if log_domain else np.float64(out[p, o])
            assert abs(got_out - v[rest].max()) <= REL * v[rest].max() + ABS
    _compare(farm, mem, ws, qb, cfg.k, dtype)


def test_default_form_256_queries_full_size(farm):
    """The benchmark's default form at its full size and launch shape: BF16
    similarities and learned proposals from the benchmark's own trained
    network, 4,096 queries over N = 20,000 objects in one call; a fixed subset
    of 256 queries against the oracle's exact TopK, with the winners'
    per-relation terms."""
    import bench
    from tests import _gpu
    from tests._parity import TOPK_FLOOR
    from tests.test_gpu_parity import _check_bounded
    cfg = CONFIGS["precision"]
    scene = make_scene(cfg)
    qb = make_queries(cfg, scene)
    mem = _gpu.build_memory(scene, flags=farm.FARM_BUILD_BF16 | farm.FARM_BUILD_FP8)
    args = bench.parse([])
    net = bench.train_network(farm, cfg, args)
    farm.build_proposals(mem, net, args.list_m)
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 64)
    print(f"[default form] n={scene.n} q={qb.q} R={qb.r_tot}", flush=True)
    ids, sc, terms, anch, cert = _gpu.query_topk(mem, ws, qb, cfg.k, dtype=farm.BF16, with_cert=True,
                                                 method=farm.PROPOSAL)
    assert np.all(cert == 1)
    rows = np.sort(np.random.default_rng(2606).choice(qb.q, size=256, replace=False))
    sub = qb.subset(rows)
    oidx, osc, ot, ob, ns = oracle.topk_bounded(scene, sub, cfg.k + 6)
    assert np.all(osc[:, :cfg.k] >= TOPK_FLOOR)  # pure relative tolerance on every returned score
    _check_bounded(scene, sub, ids[rows], sc[rows], oidx, osc, cfg.k)
    from tests._parity import assert_values_close
    for row, qq in enumerate(rows):
        r = int(qb.rel_off[qq + 1] - qb.rel_off[qq])
        for rank in range(cfg.k):
            if int(ids[qq, rank]) == int(scene.ids[oidx[row, rank]]):
                assert_values_close(terms[qq, rank, :r], ot[row, rank, :r], "winner terms")
