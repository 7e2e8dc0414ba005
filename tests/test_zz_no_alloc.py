"""farm_query_topk_static (no workspace, no allocation) against farm_query_topk.

The allocation-free entry point lays its scratch out in the library's static
device array.  Its results must equal those of the workspace entry point on
the same inputs (ids exactly; scores, terms and bound anchors to the FP32
bar), on two calls in a row with the second one smaller (the array keeps the
first call's contents), for the exhaustive, bound-pruned and learned-proposal
methods; a call too large for the array is refused with a clear error.
"""
import numpy as np
import pytest

from synth import CONFIGS, make_queries, make_scene
from tests._parity import REL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def farm():
    import paper_2606_15476_amd as farm
    return farm


def _run(farm, fn, mem, qb, k, **kw):
    import torch
    from tests import _gpu
    target, anchors = _gpu.query_tensors(qb)
    q = qb.q
    dev = _gpu.device()
    oid = torch.full((q, k), -7, dtype=torch.int32, device=dev)
    osc = torch.full((q, k), np.nan, dtype=torch.float32, device=dev)
    ot = torch.full((q, k, 8), np.nan, dtype=torch.float32, device=dev)
    ob = torch.full((q, k, 8), -7, dtype=torch.int32, device=dev)
    cert = torch.full((q,), -1, dtype=torch.int32, device=dev)
    fn(mem, target, qb.target_cls, qb.rel_off, qb.rel_pred, anchors, k, oid, osc, ot, ob, certified=cert, **kw)
    torch.cuda.synchronize()
    return (oid.cpu().numpy().view(np.uint32), osc.cpu().numpy(), ot.cpu().numpy(),
            ob.cpu().numpy().view(np.uint32), cert.cpu().numpy())


def _with_ws(farm, ws):
    def call(mem, *a, **kw):
        farm.query_topk(mem, ws, *a, **kw)
    return call


def _same(a, b, what):
    ids_a, sc_a, t_a, b_a, c_a = a
    ids_b, sc_b, t_b, b_b, c_b = b
    np.testing.assert_array_equal(ids_a, ids_b, err_msg=f"{what}: ids")
    np.testing.assert_array_equal(b_a, b_b, err_msg=f"{what}: bound anchors")
    np.testing.assert_array_equal(c_a, c_b, err_msg=f"{what}: certificates")
    fin = np.isfinite(sc_b)
    assert np.array_equal(fin, np.isfinite(sc_a)), what
    assert np.all(np.abs(sc_a[fin] - sc_b[fin]) <= REL * np.abs(sc_b[fin])), f"{what}: scores"
    assert np.all(np.abs(t_a - t_b) <= REL * np.abs(t_b)), f"{what}: terms"


@pytest.mark.parametrize("dtype,method", [(0, 0), (1, 0), (1, 1), (1, 2), (0, 2)],
                         ids=["f32-exhaustive", "bf16-exhaustive", "bf16-bounded", "bf16-proposal", "f32-proposal"])
def test_static_equals_workspace_two_calls(farm, dtype, method):
    from tests import _gpu
    cfg = CONFIGS["mid"]
    big = make_scene(cfg, n=3000, seed=61)
    small = make_scene(cfg, n=700, seed=62)
    print(f"[static] dtype={dtype} method={method} n={big.n}, then n={small.n}", flush=True)
    runs = []
    for scene, q, seed in ((big, 40, 63), (small, 6, 64)):
        qb = make_queries(cfg, scene, seed=seed, q=q)
        mem = _gpu.build_memory(scene, flags=farm.FARM_BUILD_BF16)
        if method == farm.PROPOSAL:
            farm.build_proposals(mem, farm.ProposalNet(scene.d, max_batch=256, seed=3), 32)
        runs.append((scene, qb, mem))
    outs = []
    for scene, qb, mem in runs:  # both static calls first: the second finds the first's contents
        outs.append(_run(farm, farm.query_topk_static, mem, qb, 10, dtype=dtype, method=method))
    for (scene, qb, mem), got in zip(runs, outs):
        ws = farm.Workspace(mem, qb.q, qb.r_tot, 64)
        want = _run(farm, _with_ws(farm, ws), mem, qb, 10, dtype=dtype, method=method)
        _same(got, want, f"n={scene.n} q={qb.q}")


def test_static_tiny_and_limits(farm):
    import torch
    from tests import _gpu
    cfg = CONFIGS["tiny"]
    scene = make_scene(cfg)
    qb = make_queries(cfg, scene)
    mem = _gpu.build_memory(scene)
    ws = farm.Workspace(mem, qb.q, qb.r_tot, 16)
    got = _run(farm, farm.query_topk_static, mem, qb, 10)
    want = _run(farm, _with_ws(farm, ws), mem, qb, 10)
    _same(got, want, "tiny")
    # a call whose layout does not fit the static array is refused, and the next one still works
    big = make_scene(CONFIGS["precision"], n=20000, seed=65)
    bqb = make_queries(CONFIGS["precision"], big, seed=66, q=512)
    bmem = _gpu.build_memory(big)
    target, anchors = _gpu.query_tensors(bqb)
    oid = torch.empty((bqb.q, 10), dtype=torch.int32, device=_gpu.device())
    osc = torch.empty((bqb.q, 10), dtype=torch.float32, device=_gpu.device())
    with pytest.raises(farm.FarmError) as e:
        farm.query_topk_static(bmem, target, bqb.target_cls, bqb.rel_off, bqb.rel_pred, anchors, 10, oid, osc)
    assert e.value.status == -1 and "static scratch" in str(e.value)
    got = _run(farm, farm.query_topk_static, mem, qb, 10)
    _same(got, want, "tiny after a refused call")
