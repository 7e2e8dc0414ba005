"""Multi-channel reciprocal-rank fusion of the unary scores on the GPU against the FP64 oracle
(oracle/rrf.py), through the C ABI.

  * the fused rows (targets and anchors) element by element: within the values the exact ranks
    give, or -- where two cosines lie within 4e-6 of each other, so that FP32 cosines may order
    them either way -- between the values of the smallest and largest ranks those near-ties allow;
  * TopK of the exhaustive, bound-pruned and proposal methods against the oracle's scores with
    the fused rows (the same tie-aware interval);
  * exact ties (identical embeddings) ranked by id; the entry points' checks.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import rrf
from synth import CONFIGS, make_queries, make_scene
from tests._parity import REL, assert_values_close, assert_values_within
from tests.test_gpu_parity import _check_topk_rows

pytestmark = pytest.mark.gpu

EPS = 4e-6


@pytest.fixture(scope="module")
def farm():
    import paper_2606_15476_amd as farm
    return farm


def _world(seed, n=1500, q=24):
    cfg = CONFIGS["mid"]
    scene = make_scene(cfg, n=n, seed=seed)
    qb = make_queries(cfg, scene, seed=seed + 1, q=q, r_min=0, r_max=3)
    qb.target_cls[::4] = -1
    spaces, tv, av = synth.add_embedding_spaces(cfg, scene, qb, seed=seed + 2)
    # four channels over three spaces, weights 1.0 / 0.5 / 0.75 / 1.0: the descriptor space with the
    # target vector and with a noisier one (standing in for the raw utterance), then the other two
    rng = np.random.default_rng(seed + 3)
    noisy_t = qb.target + rng.standard_normal(qb.target.shape).astype(np.float32) * 0.01
    noisy_a = qb.rel_anchor + rng.standard_normal(qb.rel_anchor.shape).astype(np.float32) * 0.01
    channels = [(0, 1.0, qb.target, qb.rel_anchor), (0, 0.5, noisy_t, noisy_a), (1, 0.75, tv[0], av[0]),
                (2, 1.0, tv[1], av[1])]
    return cfg, scene, qb, [scene.desc] + spaces, channels


def _device_channels(farm, mem, spaces, channels):
    import torch
    from tests import _gpu
    for sp in spaces[1:]:
        mem.add_embedding_space(_gpu.to_dev(sp))
    return [(s, w, _gpu.to_dev(t), _gpu.to_dev(a) if a.size else None) for s, w, t, a in channels]


def _oracle_rows(scene, qb, spaces, channels, mode=0):
    tch = [(s, w, t) for s, w, t, _ in channels]
    ach = [(s, w, a) for s, w, _, a in channels]
    return rrf.similarities(scene, [np.asarray(x, np.float64) for x in spaces], tch, ach, qb.target_cls, mode,
                            EPS if mode else 0.0)


@pytest.mark.parametrize("seed,n", [(61, 1500), (65, 26000)])
def test_fused_rows_elementwise(farm, seed, n):
    """n = 1,500: rows ranked in LDS; n = 26,000: rows too long for LDS, ranked through global scratch.
    The long case also plants exact ties: 200 objects whose embeddings in the second space copy those
    of 200 others, so their cosines are equal and only the ids order them."""
    import torch
    from tests import _gpu
    cfg, scene, qb, spaces, channels = _world(seed, n=n, q=24 if n < 20000 else 6)
    if n > 20000:
        spaces[1][200:400] = spaces[1][0:200]
    mem = _gpu.build_memory(scene)
    dch = _device_channels(farm, mem, spaces, channels)
    ws = farm.Workspace(mem, qb.q, max(qb.r_tot, 1), 16)
    out = torch.empty((qb.q + qb.r_tot, scene.n), dtype=torch.float32, device="cuda")
    farm.rrf_similarity(mem, ws, dch, qb.target_cls, qb.rel_off, qb.rel_pred, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy().astype(np.float64)
    sem, asim = _oracle_rows(scene, qb, spaces, channels)
    lo_s, lo_a = _oracle_rows(scene, qb, spaces, channels, -1)
    hi_s, hi_a = _oracle_rows(scene, qb, spaces, channels, +1)
    ref, lo, hi = np.vstack([sem, asim]), np.vstack([lo_s, lo_a]), np.vstack([hi_s, hi_a])
    assert np.all(lo <= ref + 1e-15) and np.all(ref <= hi + 1e-15)
    assert_values_within(got, lo, hi, "fused rows")
    exact = lo == hi
    print(f"rows {got.shape}, elements with an open near-tie: {int((~exact).sum())}", flush=True)
    assert_values_close(got[exact], ref[exact], "fused rows (no near-tie)", rel=REL, abs_=0.0)


@pytest.mark.parametrize("method", ["exhaustive", "bounded", "proposal"])
def test_fused_topk(farm, method):
    from tests import _gpu
    import torch
    cfg, scene, qb, spaces, channels = _world(63)
    mem = _gpu.build_memory(scene)
    dch = _device_channels(farm, mem, spaces, channels)
    ws = farm.Workspace(mem, qb.q, max(qb.r_tot, 1), 16)
    m = {"exhaustive": farm.EXHAUSTIVE, "bounded": farm.BOUNDED, "proposal": farm.PROPOSAL}[method]
    if method == "proposal":
        farm.build_proposals(mem, farm.ProposalNet(scene.d, max_batch=4096, seed=3), 32)
    k = cfg.k
    oid = torch.empty((qb.q, k), dtype=torch.int32, device="cuda")
    osc = torch.empty((qb.q, k), dtype=torch.float32, device="cuda")
    cert = torch.zeros(qb.q, dtype=torch.int32, device="cuda")
    farm.query_topk_rrf(mem, ws, dch, qb.target_cls, qb.rel_off, qb.rel_pred, k, oid, osc, certified=cert,
                        method=m)
    torch.cuda.synchronize()
    ids, sc = oid.cpu().numpy().view(np.uint32), osc.cpu().numpy()
    assert np.all(cert.cpu().numpy() == 1)
    full = []
    for mode in (0, -1, 1):
        sem, asim = _oracle_rows(scene, qb, spaces, channels, mode)
        with oracle.similarities(sem, asim):
            full.append(oracle.score(scene, qb))
    _check_topk_rows(scene, ids, sc, tuple(full), k)


def test_equal_embeddings_rank_by_id_and_checks(farm):
    import torch
    from tests import _gpu
    cfg = CONFIGS["tiny"]
    scene = make_scene(cfg, n=50, seed=71)
    qb = make_queries(cfg, scene, seed=72, q=6, r_min=1, r_max=2)
    rng = np.random.default_rng(5)
    sp1 = rng.standard_normal((scene.n, 16)).astype(np.float32)
    sp1[10:20] = sp1[10]          # ten entities with one embedding: equal cosines, ranked by id
    sp1[30:33] = 2.5 * sp1[30]    # equal after normalisation too
    channels = [(0, 1.0, qb.target, qb.rel_anchor),
                (1, 0.75, rng.standard_normal((qb.q, 16)).astype(np.float32),
                 rng.standard_normal((qb.r_tot, 16)).astype(np.float32))]
    spaces = [scene.desc, sp1]
    mem = _gpu.build_memory(scene)
    dch = _device_channels(farm, mem, spaces, channels)
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 16)
    out = torch.empty((qb.q + qb.r_tot, scene.n), dtype=torch.float32, device="cuda")
    farm.rrf_similarity(mem, ws, dch, qb.target_cls, qb.rel_off, qb.rel_pred, out)
    torch.cuda.synchronize()
    sem, asim = _oracle_rows(scene, qb, spaces, channels)
    lo = np.vstack(_oracle_rows(scene, qb, spaces, channels, -1))
    hi = np.vstack(_oracle_rows(scene, qb, spaces, channels, +1))
    assert_values_within(out.cpu().numpy().astype(np.float64), lo, hi, "fused rows with exact ties")
    # checks: reduced precision, unknown space, non-positive weight, an invalid space
    oid = torch.empty((qb.q, 4), dtype=torch.int32, device="cuda")
    osc = torch.empty((qb.q, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(farm.FarmError) as e:
        farm.query_topk_rrf(mem, ws, dch, qb.target_cls, qb.rel_off, qb.rel_pred, 4, oid, osc, dtype=farm.BF16)
    assert e.value.status == -4
    for bad in ([(5,) + tuple(dch[1][1:])], [(1, 0.0) + tuple(dch[1][2:])], [(1, float("nan")) + tuple(dch[1][2:])]):
        with pytest.raises(farm.FarmError) as e:
            farm.rrf_similarity(mem, ws, bad, qb.target_cls, qb.rel_off, qb.rel_pred, out)
        assert e.value.status == -1
    zero = np.array(sp1)
    zero[3] = 0.0
    with pytest.raises(farm.FarmError) as e:
        mem.add_embedding_space(_gpu.to_dev(zero))
    assert e.value.status == -1
