"""The proposal network's GPU kernels against the FP64 oracle.

  * inputs: the BF16 input rows equal the oracle's features (descriptors and the
    12 relative-geometry values / 4 m) up to BF16 rounding;
  * gradients: the GPU's backward pass on a batch equals the oracle's FP64
    backward on the very same BF16-rounded inputs and weights, to the accuracy
    of BF16 activations (relative error of each gradient tensor < 3e-2, cosine
    > 0.999);
  * training with the project's own AdamW steps lowers the loss.
"""
import numpy as np
import pytest

import oracle
from synth import CONFIGS, make_scene

pytestmark = pytest.mark.gpu


def _bf16_round(a):
    a = np.asarray(a, np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def _bf16_to_f32(u16):
    return (np.asarray(u16, np.uint16).astype(np.uint32) << 16).view(np.float32)


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
    nb = 200
    o = rng.integers(0, scene.n, nb).astype(np.int32)
    a = rng.integers(0, scene.n, nb).astype(np.int32)
    pred = rng.integers(0, 5, nb).astype(np.int32)
    lab = rng.integers(0, 2, nb).astype(np.float32)
    dev = lambda x: torch.from_numpy(x).cuda()
    return farm, scene, mem, net, (dev(o), dev(a), dev(pred), dev(lab)), (o, a, pred, lab)


def test_inputs_match_oracle_features(setup):
    import torch
    farm, scene, mem, net, dv, hv = setup
    o, a = hv[0], hv[1]
    X = torch.zeros((len(o), net.in_dim), dtype=torch.int16, device="cuda")
    net.inputs(mem, dv[0], dv[1], X)
    torch.cuda.synchronize()
    Xf = _bf16_to_f32(X.cpu().numpy().view(np.uint16))
    d = scene.d
    dp = (d + 63) // 64 * 64
    u = scene.desc.astype(np.float64)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    for b in range(0, len(o), 17):
        np.testing.assert_allclose(Xf[b, :d], u[o[b]], rtol=2 ** -8, atol=1e-7)
        np.testing.assert_allclose(Xf[b, dp:dp + d], u[a[b]], rtol=2 ** -8, atol=1e-7)
        g = oracle.pair_features(scene, int(o[b]), int(a[b])) / 4.0
        np.testing.assert_allclose(Xf[b, 2 * dp:2 * dp + 12], g, rtol=2 ** -7, atol=1e-6)
        assert np.all(Xf[b, d:dp] == 0) and np.all(Xf[b, 2 * dp + 12:] == 0)


def test_gradients_match_oracle(setup):
    import torch
    farm, scene, mem, net, dv, hv = setup
    o, a, pred, lab = hv
    # weights as the GPU uses them: BF16-rounded W1, W2, W3
    w = net.weights()
    wr = {k: (_bf16_round(v) if k.startswith("W") else v).astype(np.float64) for k, v in w.items()}
    X = torch.zeros((len(o), net.in_dim), dtype=torch.int16, device="cuda")
    net.inputs(mem, dv[0], dv[1], X)
    loss_d = torch.zeros(1, dtype=torch.float32, device="cuda")
    net.step(mem, *dv, update=False, loss_out=loss_d)
    torch.cuda.synchronize()
    g = net.grads()
    Xf = _bf16_to_f32(X.cpu().numpy().view(np.uint16)).astype(np.float64)
    loss64, _, g64 = oracle.mlp(wr, Xf, pred, lab.astype(np.float64))
    assert float(loss_d.cpu()[0]) == pytest.approx(loss64, rel=5e-3)
    for k in net.PARAMS:
        a_, b_ = g[k].astype(np.float64).ravel(), g64[k].ravel()
        rel = np.linalg.norm(a_ - b_) / max(np.linalg.norm(b_), 1e-30)
        cos = float(a_ @ b_ / max(np.linalg.norm(a_) * np.linalg.norm(b_), 1e-30))
        print(f"grad {k}: rel err {rel:.2e}, cosine {cos:.6f}", flush=True)
        assert rel < 3e-2 and cos > 0.999, k


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
