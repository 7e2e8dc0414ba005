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
