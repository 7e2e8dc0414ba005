"""The proposal network's GPU kernels against the FP64 oracle, element by element.

  * inputs: the BF16 input rows equal the oracle's features (descriptors and the
    12 relative-geometry values / 4 m) up to BF16 rounding;
  * every layer of one training step, forward and backward, on its own stored
    inputs (oracle/mlp_layers.py): each element of Z1, A1, Z2, A2, Y, dZ2,
    dA1, dZ1 and of every gradient lies within the bound that FP32
    accumulation and BF16 storage allow; the batch covers all nine outputs and
    pairs of predicates without an output (which add nothing);
  * end to end: the GPU gradients against the oracle's own FP64 chain from the
    same inputs and weights (BF16 activations then differ by up to 2^-8 per
    layer: checked as tensor-wise relative error and cosine);
  * AdamW: two steps, each weight element against the oracle's FP64 update
    from the GPU's gradients;
  * the table build's factorised forward and the plain forward: each logit of
    every anchor of sampled targets within the oracle's forward bound; each
    list is exactly the top M of the table's logits;
  * training with the project's own AdamW steps lowers the loss.
"""
import numpy as np
import pytest

import oracle
from oracle import mlp_layers as ml
from synth import CONFIGS, make_scene

pytestmark = pytest.mark.gpu


def _bf16_round(a):
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def _bf16_to_f64(u16):
    return (np.asarray(u16, np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _weights_as_used(net):
    w = net.weights()
    return {k: (_bf16_round(v) if k.startswith("W") else v).astype(np.float64) for k, v in w.items()}


def _assert_within(got, ref, tol, what):
    got = np.asarray(got, np.float64)
    err = np.abs(got - ref)
    bad = err > tol
    worst = float(np.max(err / np.maximum(tol, 1e-300)))
    print(f"{what}: max err / bound {worst:.3g}", flush=True)
    if bad.any():
        i = np.unravel_index(np.argmax(err - tol), err.shape)
        raise AssertionError(f"{what}: {int(bad.sum())} of {bad.size} outside the bound; worst at {i}: "
                             f"got {got[i]!r} ref {ref[i]!r} bound {tol[i]:.3g}")


@pytest.fixture(scope="module")
def setup():
    import torch
    import paper_2606_15476_amd as farm
    from tests import _gpu
    cfg = CONFIGS["mid"]
    scene = make_scene(cfg, n=300, seed=5)
    mem = _gpu.build_memory(scene)
    net = farm.ProposalNet(scene.d, max_batch=512, seed=3)
    rng = np.random.default_rng(0)
    nb = 230
    o = rng.integers(0, scene.n, nb).astype(np.int32)
    a = rng.integers(0, scene.n, nb).astype(np.int32)
    pred = rng.integers(0, 12, nb).astype(np.int32)  # 9..11 have no output
    pred[:9] = np.arange(9)
    lab = rng.integers(0, 2, nb).astype(np.float32)
    dev = lambda x: torch.from_numpy(x).cuda()
    return farm, scene, mem, net, (dev(o), dev(a), dev(pred), dev(lab)), (o, a, pred, lab)


def _inputs(net, mem, o_t, a_t):
    import torch
    X = torch.zeros((int(o_t.shape[0]), net.in_dim), dtype=torch.int16, device="cuda")
    net.inputs(mem, o_t, a_t, X)
    torch.cuda.synchronize()
    return _bf16_to_f64(X.cpu().numpy().view(np.uint16))


def test_inputs_match_oracle_features(setup):
    farm, scene, mem, net, dv, hv = setup
    o, a = hv[0], hv[1]
    Xf = _inputs(net, mem, dv[0], dv[1])
    d = scene.d
    dp = (d + 63) // 64 * 64
    u = scene.desc.astype(np.float64)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    for b in range(len(o)):
        np.testing.assert_allclose(Xf[b, :d], u[o[b]], rtol=2 ** -8, atol=1e-7)
        np.testing.assert_allclose(Xf[b, dp:dp + d], u[a[b]], rtol=2 ** -8, atol=1e-7)
        g = oracle.pair_features(scene, int(o[b]), int(a[b])) / 4.0
        np.testing.assert_allclose(Xf[b, 2 * dp:2 * dp + 12], g, rtol=2 ** -7, atol=1e-6)
        assert np.all(Xf[b, d:dp] == 0) and np.all(Xf[b, 2 * dp + 12:] == 0)


@pytest.fixture(scope="module")
def one_step(setup):
    """One forward/backward step (no update): inputs, weights, stored stage tensors, loss, gradients."""
    import torch
    farm, scene, mem, net, dv, hv = setup
    W = _weights_as_used(net)
    X = _inputs(net, mem, dv[0], dv[1])
    loss_d = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.step(mem, *dv, update=False, loss_out=loss_d)
    torch.cuda.synchronize()
    nb = X.shape[0]
    b = net.batch(nb)
    st = {k: (_bf16_to_f64(v) if v.dtype == np.uint16 else v.astype(np.float64)) for k, v in b.items()}
    return W, X, st, float(loss_d.cpu()[0]), net.grads()


def test_forward_layers_elementwise(setup, one_step):
    W, X, st, _, _ = one_step
    refs = ml.forward_stages(W, X, st)
    for name in ("Z1", "A1", "Z2", "A2", "Y"):
        ref, tol = refs[name]
        _assert_within(st[name], ref, tol, name)


def test_backward_layers_and_gradients_elementwise(setup, one_step):
    farm, scene, mem, net, dv, hv = setup
    W, X, st, loss, g = one_step
    pred, lab = hv[2], hv[3].astype(np.float64)
    refs = ml.backward_stages(W, X, st, pred, lab)
    ref, tol = refs["loss"]
    assert abs(loss - ref) <= tol + 1e-7, (loss, ref)
    for name in ("dZ2", "dA1", "dZ1"):
        _assert_within(st[name], *refs[name], name)
    for k in net.PARAMS:
        _assert_within(g[k], *refs["g" + k], "grad " + k)
    # every output received a gradient; the pairs without an output left the
    # rows of dZ2 zero
    assert np.all(np.abs(g["b3"]) > 0)
    assert np.all(st["dZ2"][pred >= 9] == 0)


def test_end_to_end_gradients_match_oracle(setup, one_step):
    """The oracle's own FP64 chain from the same inputs and weights: the GPU's
    BF16 activations move each tensor by well under 3e-2 of its norm."""
    farm, scene, mem, net, dv, hv = setup
    W, X, st, loss, g = one_step
    o, a, pred, lab = hv
    keep = pred < oracle.NPRED
    loss64, _, g64 = oracle.mlp(W, X[keep], pred[keep], lab[keep].astype(np.float64))
    scale = keep.sum() / len(pred)
    assert loss == pytest.approx(loss64 * scale, rel=5e-3)
    for k in net.PARAMS:
        a_, b_ = g[k].astype(np.float64).ravel(), g64[k].ravel() * scale
        rel = np.linalg.norm(a_ - b_) / max(np.linalg.norm(b_), 1e-30)
        cos = float(a_ @ b_ / max(np.linalg.norm(a_) * np.linalg.norm(b_), 1e-30))
        print(f"grad {k}: rel err {rel:.2e}, cosine {cos:.6f}", flush=True)
        assert rel < 3e-2 and cos > 0.999, k


def test_adamw_two_steps_elementwise(setup):
    farm, scene, mem, net0, dv, hv = setup
    net = farm.ProposalNet(scene.d, max_batch=512, seed=9)
    lr, wd = 2e-3, 1e-2
    w_prev = net.weights()
    m = {k: np.zeros(v.shape) for k, v in w_prev.items()}
    v = {k: np.zeros(v.shape) for k, v in w_prev.items()}
    for step in (1, 2):
        net.step(mem, *dv, lr=lr, weight_decay=wd, update=True)
        g = net.grads()
        w_now = net.weights()
        for k in net.PARAMS:
            ref, m[k], v[k], tol = ml.adamw(w_prev[k], g[k], m[k], v[k], step, lr, wd)
            _assert_within(w_now[k], ref, tol, f"AdamW step {step} {k}")
        w_prev = w_now


def test_table_and_plain_logits_elementwise(setup):
    """The factorised forward of the table build and the plain forward, every
    anchor of three targets, each logit within the oracle's forward bound; the
    lists are the top M of the table's logits."""
    import torch
    farm, scene, mem, net0, dv, hv = setup
    net = farm.ProposalNet(scene.d, max_batch=512, seed=13)
    net.step(mem, *dv, lr=3e-3, update=True)  # away from the initialisation
    W = _weights_as_used(net)
    n, P, t0, tc, M = scene.n, oracle.NPRED, 17, 3, 40
    L = torch.empty((P, tc, n), dtype=torch.float32, device="cuda")
    net.table_logits(mem, t0, tc, L)
    L = L.cpu().numpy().astype(np.float64)
    farm.build_proposals(mem, net, M)
    _, idx, _, _ = farm.get_proposals(mem)
    idx = idx.cpu().numpy()
    for t in range(tc):
        o = t0 + t
        o_t = torch.full((n,), o, dtype=torch.int32, device="cuda")
        a_t = torch.arange(n, dtype=torch.int32, device="cuda")
        X = _inputs(net, mem, o_t, a_t)
        y, bound = ml.forward_bound(W, X)
        others = np.arange(n) != o
        assert np.all(np.isneginf(L[:, t, o]))
        _assert_within(L[:, t, others].T, y[others], bound[others], f"table logits target {o}")
        plain = torch.empty((n, P), dtype=torch.float32, device="cuda")
        net.logits(mem, o_t, a_t, plain)
        torch.cuda.synchronize()
        _assert_within(plain.cpu().numpy()[others], y[others], bound[others], f"plain logits target {o}")
        for p in range(P):
            on = np.zeros(n, bool)
            on[idx[p, o]] = True
            assert on.sum() == M and not on[o]
            assert L[p, t, on].min() >= L[p, t, ~on & others].max(), (o, p)


def test_training_lowers_the_loss(setup):
    import torch
    farm, scene, mem, net2, dv, hv = setup
    net = farm.ProposalNet(scene.d, max_batch=512, seed=11)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for it in range(60):
        net.step(mem, *dv, lr=3e-3, weight_decay=0.0, update=True, loss_out=loss)
        hist.append(float(loss.cpu()[0]))
    print(f"loss {hist[0]:.4f} -> {hist[-1]:.4f}", flush=True)
    assert hist[-1] < 0.5 * hist[0]
