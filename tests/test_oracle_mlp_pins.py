"""Pins for the oracle's proposal network (FP64): closed forms of GELU and the
BCE loss, hand-computed pair features, and central finite differences of
every gradient on a small network."""
import math

import numpy as np
import pytest

import oracle
from synth import Scene

NP = oracle.NPRED  # one network output per predicate


def _weights(rng, inp, h, scale=0.3):
    return {"W1": rng.standard_normal((h, inp)) * scale, "b1": rng.standard_normal(h) * 0.1,
            "W2": rng.standard_normal((h, h)) * scale, "b2": rng.standard_normal(h) * 0.1,
            "W3": rng.standard_normal((NP, h)) * scale, "b3": rng.standard_normal(NP) * 0.1}


def test_zero_network_closed_forms():
    """All weights zero: y = b3, so the loss is the BCE of a constant logit."""
    inp, h = 7, 4
    W = {k: np.zeros_like(v) for k, v in _weights(np.random.default_rng(0), inp, h).items()}
    W["b3"] = np.array([0.0, 1.0, -2.0, 0.5, 3.0, -1.0, 0.25, 2.0, -0.5])
    X = np.ones((6, inp))
    pred = np.array([0, 1, 2, 4, 5, 8], np.int32)
    lab = np.array([1.0, 0.0, 1.0, 1.0, 0.0, 1.0])
    loss, logits, g = oracle.mlp(W, X, pred, lab)
    sp = lambda v: math.log1p(math.exp(v))  # softplus
    # BCE(y, t) = softplus(y) - t y
    want = (math.log(2.0) + sp(1.0) + sp(2.0) + sp(-3.0) + sp(-1.0) + sp(0.5)) / 6.0
    assert loss == pytest.approx(want, rel=1e-14)
    np.testing.assert_array_equal(logits, np.tile(W["b3"], (6, 1)))
    # d loss / d b3[p] = mean over samples with that predicate of sigmoid(y) - label
    sig = lambda v: 1 / (1 + math.exp(-v))
    assert g["b3"][0] == pytest.approx((sig(0.0) - 1) / 6)
    assert g["b3"][1] == pytest.approx(sig(1.0) / 6)
    assert g["b3"][5] == pytest.approx(sig(-1.0) / 6)
    assert g["b3"][8] == pytest.approx((sig(-0.5) - 1) / 6)
    assert g["b3"][3] == 0.0 and g["b3"][6] == 0.0 and g["b3"][7] == 0.0


def test_gelu_values_through_a_one_unit_network():
    """h = 1, identity-like weights expose GELU(z) in the logit: y = GELU(GELU(z))."""
    inp, h = 1, 1
    W = {"W1": np.array([[1.0]]), "b1": np.zeros(1), "W2": np.array([[1.0]]), "b2": np.zeros(1),
         "W3": np.ones((NP, 1)), "b3": np.zeros(NP)}
    gelu = lambda v: 0.5 * v * (1 + math.erf(v / math.sqrt(2)))
    for z, g1 in ((0.0, 0.0), (1.0, 0.8413447460685429), (-1.0, -0.15865525393145707)):
        assert gelu(z) == pytest.approx(g1, abs=1e-15)
        _, logits, _ = oracle.mlp(W, np.array([[z]]), np.zeros(1, np.int32), np.zeros(1), grads=False)
        assert logits[0, 0] == pytest.approx(gelu(g1), abs=1e-15)


def test_pair_features_hand_computed():
    center = np.array([[1.0, 2.0, 3.0], [0.5, -1.0, 1.0]], np.float32)
    extent = np.array([[0.2, 0.4, 1.0], [2.0, 1.0, 0.5]], np.float32)
    scene = Scene(desc=np.ones((2, 4), np.float32), center=center, extent=extent,
                  ids=np.array([1, 2], np.uint32), cls=np.zeros(2, np.int32),
                  view_right=np.array([0.6, 0.8], np.float32), centroids=np.zeros((1, 4), np.float32))
    g = oracle.pair_features(scene, 0, 1)
    d = np.array([0.5, 3.0, 2.0])
    want = np.concatenate([d, [0.2, 0.4, 1.0], [2.0, 1.0, 0.5],
                           [math.sqrt(0.25 + 9 + 4)], [0.5 * 0.6 + 3.0 * 0.8],
                           [(3.0 - 0.5) - (1.0 + 0.25)]])
    np.testing.assert_allclose(g, want, rtol=1e-6, atol=1e-6)


def test_gradients_match_central_differences():
    rng = np.random.default_rng(7)
    inp, h, n = 2 * 8 + 12, 16, 9
    W = _weights(rng, inp, h)
    X = rng.standard_normal((n, inp))
    pred = rng.integers(0, NP, n).astype(np.int32)
    lab = rng.integers(0, 2, n).astype(np.float64)
    loss, _, g = oracle.mlp(W, X, pred, lab)
    eps = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = W[name].reshape(-1)
        idx = rng.choice(flat.size, size=min(flat.size, 25), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + eps
            lp, _, _ = oracle.mlp(W, X, pred, lab, grads=False)
            flat[i] = old - eps
            lm, _, _ = oracle.mlp(W, X, pred, lab, grads=False)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            assert g[name].reshape(-1)[i] == pytest.approx(fd, rel=1e-5, abs=1e-9), (name, i)


# ---------------------------------------------------------------- layer-by-layer references (oracle/mlp_layers.py)
def _fp64_chain(W, X, pred, lab):
    """Stage values of an exact FP64 evaluation (what the layer references
    consume when no rounding happened)."""
    from oracle import mlp_layers as ml
    z1 = X @ W["W1"].T + W["b1"]
    a1 = ml.gelu(z1)
    z2 = a1 @ W["W2"].T + W["b2"]
    a2 = ml.gelu(z2)
    y = a2 @ W["W3"].T + W["b3"]
    _, dY, _ = ml.loss_and_dy(y, pred, lab)
    dz2 = (dY @ W["W3"]) * ml.gelu_grad(z2)
    da1 = dz2 @ W["W2"]
    dz1 = da1 * ml.gelu_grad(z1)
    return {"Z1": z1, "A1": a1, "Z2": z2, "A2": a2, "Y": y, "dZ2": dz2, "dA1": da1, "dZ1": dz1}


def test_layer_references_equal_the_loop_oracle():
    """Fed the exact FP64 stage values, the layer references reproduce the C
    oracle's plain-loop forward, loss and every gradient (two independent
    implementations); predicates without an output (9..11) add nothing."""
    from oracle import mlp_layers as ml
    rng = np.random.default_rng(4)
    inp, h, nb = 11, 6, 40
    W = _weights(rng, inp, h)
    X = rng.standard_normal((nb, inp))
    pred = rng.integers(0, 12, nb).astype(np.int32)
    lab = rng.integers(0, 2, nb).astype(np.float64)
    # the C oracle takes every sample's predicate as an output index: give it only the labelled rows,
    # scaled to the mean over all nb rows
    keep = pred < NP
    loss_c, logits_c, g_c = oracle.mlp(W, X[keep], pred[keep], lab[keep])
    scale = keep.sum() / nb
    st = _fp64_chain(W, X, pred, lab)
    fw = ml.forward_stages(W, X, st)
    np.testing.assert_allclose(fw["Y"][0][keep], logits_c, rtol=1e-12, atol=1e-14)
    for name in ("Z1", "A1", "Z2", "A2", "Y"):
        np.testing.assert_allclose(fw[name][0], st[name], rtol=1e-12, atol=1e-14)
    bw = ml.backward_stages(W, X, st, pred, lab)
    assert bw["loss"][0] == pytest.approx(loss_c * scale, rel=1e-12)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        np.testing.assert_allclose(bw["g" + k][0], g_c[k] * scale, rtol=1e-10, atol=1e-15)


def test_gelu_derivative_by_central_differences():
    from oracle import mlp_layers as ml
    v = np.linspace(-6, 6, 97)
    h = 1e-6
    fd = (ml.gelu(v + h) - ml.gelu(v - h)) / (2 * h)
    np.testing.assert_allclose(ml.gelu_grad(v), fd, rtol=1e-7, atol=1e-9)
    assert np.max(np.abs(ml.gelu_grad(np.linspace(-10, 10, 20001)))) <= ml.GELU_SLOPE_MAX


def test_forward_bound_covers_an_fp32_bf16_evaluation():
    """An explicit evaluation with FP32 products/sums and BF16-stored
    activations (numpy float32, round-to-nearest-even to 8 significant bits)
    lies within forward_bound of the FP64 logits."""
    from oracle import mlp_layers as ml

    def bf16(a):
        u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
        return u.astype(np.uint32).view(np.float32)

    rng = np.random.default_rng(6)
    inp, h, nb = 80, 64, 50
    W = {k: (bf16(v).astype(np.float64) if k.startswith("W") else v) for k, v in _weights(rng, inp, h, 0.2).items()}
    X = bf16(rng.standard_normal((nb, inp))).astype(np.float64)
    f = {k: v.astype(np.float32) for k, v in W.items()}
    g32 = lambda z: (np.float32(0.5) * z * (np.float32(1) + erf_f32(z / np.float32(math.sqrt(2))))).astype(np.float32)
    a1 = bf16(g32(X.astype(np.float32) @ f["W1"].T + f["b1"]))
    a2 = bf16(g32(a1 @ f["W2"].T + f["b2"]))
    y32 = a2 @ f["W3"].T + f["b3"]
    y, bound = ml.forward_bound(W, X)
    err = np.abs(y32.astype(np.float64) - y)
    assert np.all(err <= bound), float(np.max(err / bound))
    assert np.max(err / bound) > 1e-3  # the bound is not vacuous


def erf_f32(z):
    from scipy.special import erf
    return erf(z.astype(np.float64)).astype(np.float32)


def test_adamw_reference():
    """Step 1 from zero moments: m_hat = g, v_hat = g^2, so the step is
    lr (g / (|g| + eps) + wd w); two steps equal torch.optim.AdamW (float64)."""
    import torch
    from oracle import mlp_layers as ml
    rng = np.random.default_rng(8)
    w = rng.standard_normal(50)
    g1 = rng.standard_normal(50) * 1e-2
    g1[:3] = [0.0, 1e-12, -1e-9]
    lr, wd = 2e-3, 1e-4
    w1, m1, v1, _ = ml.adamw(w, g1, np.zeros(50), np.zeros(50), 1, lr, wd)
    np.testing.assert_allclose(w1, w - lr * (g1 / (np.abs(g1) + 1e-8) + wd * w), rtol=1e-13, atol=1e-16)
    g2 = rng.standard_normal(50) * 1e-2
    w2, _, _, _ = ml.adamw(w1, g2, m1, v1, 2, lr, wd)
    p = torch.nn.Parameter(torch.tensor(w, dtype=torch.float64))
    opt = torch.optim.AdamW([p], lr=lr, betas=(0.9, 0.999), eps=1e-8, weight_decay=wd)
    for g in (g1, g2):
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    np.testing.assert_allclose(w2, p.detach().numpy(), rtol=1e-12, atol=1e-15)
