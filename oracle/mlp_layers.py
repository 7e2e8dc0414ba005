"""Layer-by-layer FP64 references of the anchor proposal network.

TEST INFRASTRUCTURE ONLY (like the rest of ``oracle/``): only the test suite may
import it.  It shares no code with the GPU library.

The network is not a construct of the paper: it produces the anchor candidate
sets K_a of the query-time complexity analysis (Appendix "Robust Relational
Retrieval Formulation").  Its definition (the library header's proposal-network
section):

    x  = [u_o ; u_a ; g(o, a) / 4 m ; 0]
    h1 = GELU(W1 x + b1),  h2 = GELU(W2 h1 + b2),  y = W3 h2 + b3
    GELU(v) = v/2 (1 + erf(v / sqrt 2))
    loss = mean_s BCEwithLogits(y_s[p_s], label_s) over pairs whose predicate
           has an output (the others count in the mean and add nothing)

with BF16 weights and BF16 stored activations (h1, h2 and the back-propagated
pre-activation gradients), FP32 accumulation.  Every function here takes the
values a stage of such an implementation consumed -- its own stored inputs --
and returns, in FP64, what that stage must produce, together with a per-element
bound on the error that its FP32 arithmetic and BF16 storage may add:

  * FP32 accumulation of K exact products (BF16 x BF16 is exact in FP32) plus
    a bias: |err| <= (K + 2) u * sum|terms|, u = 2^-24 (the classical bound of
    recursive summation; any blocking order obeys it);
  * storage in BF16 (round to nearest even): half an ulp, <= 2^-8 |value|;
  * an FP32 GELU or GELU' (erff, expf, a few products): a few ulps of the
    operands, bounded here by 8 u (|v| + |result|) -- absolute, since
    1 + erf(v) cancels for negative v.

A planted mistake (a transposed operand, a wrong derivative, a dropped bias)
moves an element by a sizeable fraction of sum|terms|, far outside these
bounds.  Plain numpy: matrix products as the library primitive, the rest
elementwise in the order of the definition.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

U32 = 2.0 ** -24   # FP32 unit roundoff
UBF = 2.0 ** -8    # BF16 unit roundoff (8-bit significand)
GELU_SLOPE_MAX = 1.13  # max |GELU'(v)| over all v (1.129 at v = sqrt 2)
NPRED = 9


def gelu(v):
    v = np.asarray(v, np.float64)
    return 0.5 * v * (1.0 + erf(v / math.sqrt(2.0)))


def gelu_grad(v):
    v = np.asarray(v, np.float64)
    return 0.5 * (1.0 + erf(v / math.sqrt(2.0))) + v * np.exp(-0.5 * v * v) / math.sqrt(2.0 * math.pi)


def _affine(A, W, b):
    """A W^T + b and the accumulation bound (K + 2) u (|A| |W|^T + |b|)."""
    ref = A @ W.T + b
    absum = np.abs(A) @ np.abs(W).T + np.abs(b)
    return ref, (A.shape[1] + 2) * U32 * absum


def _gelu_stage(Z):
    ref = gelu(Z)
    return ref, UBF * np.abs(ref) + 8 * U32 * (np.abs(Z) + np.abs(ref)) + 1e-37


def forward_stages(W, X, st):
    """Forward stages from their stored inputs.  W: FP64 weights as used
    (W1, W2, W3 BF16 values; b1, b2, b3), X [nb, in] the input rows, st: the
    stored Z1, A1, Z2, A2 (FP64 values).  Returns {name: (ref, tol)} for Z1,
    A1, Z2, A2, Y."""
    out = {"Z1": _affine(X, W["W1"], W["b1"]), "A1": _gelu_stage(st["Z1"]),
           "Z2": _affine(st["A1"], W["W2"], W["b2"]), "A2": _gelu_stage(st["Z2"]),
           "Y": _affine(st["A2"], W["W3"], W["b3"])}
    return out


def loss_and_dy(Y, pred, label, nb=None):
    """Mean BCE-with-logits on the labelled output and dL/dY, from logits Y [nb, 9]."""
    Y = np.asarray(Y, np.float64)
    nb = Y.shape[0] if nb is None else nb
    loss, dY, terms = 0.0, np.zeros_like(Y), 0.0
    for b in range(Y.shape[0]):
        p = int(pred[b])
        if not 0 <= p < NPRED:
            continue
        v, t = Y[b, p], float(label[b])
        lb = max(v, 0.0) - v * t + math.log1p(math.exp(-abs(v)))
        loss += lb
        terms += abs(max(v, 0.0)) + abs(v * t) + math.log1p(math.exp(-abs(v)))
        dY[b, p] = (1.0 / (1.0 + math.exp(-v)) - t) / nb
    return loss / nb, dY, 32 * U32 * terms / nb


def backward_stages(W, X, st, pred, label):
    """Backward stages from their stored inputs (st additionally holds dZ2,
    dA1 and dZ1 as stored).  Returns {name: (ref, tol)} for dZ2, dA1, dZ1 and
    the gradients gW3, gb3, gW2, gb2, gW1, gb1, plus the loss."""
    nb = X.shape[0]
    loss, dY, loss_tol = loss_and_dy(st["Y"], pred, label)
    # dY in FP32: a logistic, a difference and a division, a few u absolute (|sigmoid - t| <= 1)
    e_dy = 4 * U32 / nb
    out = {"loss": (loss, loss_tol)}
    dA2 = dY @ W["W3"]
    gg2 = gelu_grad(st["Z2"])
    ref = dA2 * gg2
    lab = (pred >= 0) & (pred < NPRED)
    w3row = np.zeros_like(dA2)
    w3row[lab] = np.abs(W["W3"][pred[lab]])
    out["dZ2"] = (ref, UBF * np.abs(ref) + e_dy * w3row * (np.abs(gg2) + 1.0)
                  + np.abs(dA2) * 8 * U32 * (1.0 + np.abs(st["Z2"])) + 1e-37)
    # head gradients from the FP64 dY (the stored dY is not kept): accumulation + dY's own error
    p = dY.T @ st["A2"]
    out["gW3"] = (p, (nb + 2) * U32 * (np.abs(dY).T @ np.abs(st["A2"])) + e_dy * (lab[None, :] @ np.abs(st["A2"])))
    out["gb3"] = (dY.sum(axis=0), (nb + 2) * U32 * np.abs(dY).sum(axis=0) + e_dy * lab.sum())
    # layer 2 and 1 gradients from the stored dZ2 / dZ1
    out["gW2"] = (st["dZ2"].T @ st["A1"], (nb + 2) * U32 * (np.abs(st["dZ2"]).T @ np.abs(st["A1"])))
    out["gb2"] = (st["dZ2"].sum(axis=0), (nb + 2) * U32 * np.abs(st["dZ2"]).sum(axis=0))
    out["dA1"] = (st["dZ2"] @ W["W2"], (W["W2"].shape[0] + 2) * U32 * (np.abs(st["dZ2"]) @ np.abs(W["W2"])))
    gg1 = gelu_grad(st["Z1"])
    ref = st["dA1"] * gg1
    out["dZ1"] = (ref, UBF * np.abs(ref) + np.abs(st["dA1"]) * 8 * U32 * (1.0 + np.abs(st["Z1"])) + 1e-37)
    out["gW1"] = (st["dZ1"].T @ X, (nb + 2) * U32 * (np.abs(st["dZ1"]).T @ np.abs(X)))
    out["gb1"] = (st["dZ1"].sum(axis=0), (nb + 2) * U32 * np.abs(st["dZ1"]).sum(axis=0))
    return out


def forward_bound(W, X):
    """Logits [nb, 9] of the FP64 forward pass from the input rows X, and a
    first-order bound on what an evaluation with FP32 accumulation and BF16
    stored activations (in any summation order) may differ by."""
    z1, ez1 = _affine(X, W["W1"], W["b1"])
    a1 = gelu(z1)
    ea1 = UBF * np.abs(a1) + GELU_SLOPE_MAX * ez1 + 8 * U32 * (np.abs(z1) + np.abs(a1))
    z2, ez2 = _affine(a1, W["W2"], W["b2"])
    ez2 = ez2 + ea1 @ np.abs(W["W2"]).T
    a2 = gelu(z2)
    ea2 = UBF * np.abs(a2) + GELU_SLOPE_MAX * ez2 + 8 * U32 * (np.abs(z2) + np.abs(a2))
    y, ey = _affine(a2, W["W3"], W["b3"])
    ey = ey + ea2 @ np.abs(W["W3"]).T
    return y, 1.01 * ey + 1e-6


def adamw(w, g, m, v, step, lr, wd, beta1=0.9, beta2=0.999, eps=1e-8):
    """One AdamW update (decoupled weight decay) in FP64 with exact bias
    corrections 1 - beta^step.  Returns (w', m', v', tol): tol bounds an FP32
    evaluation -- the final subtraction (2 u |w'|) and the step's relative
    error (its FP32 bias corrections alone: 1 - 0.999^t cancels, up to ~1e-4
    relative at t = 1)."""
    w, g, m, v = (np.asarray(a, np.float64) for a in (w, g, m, v))
    m1 = beta1 * m + (1.0 - beta1) * g
    v1 = beta2 * v + (1.0 - beta2) * g * g
    mh = m1 / (1.0 - beta1 ** step)
    vh = v1 / (1.0 - beta2 ** step)
    upd = mh / (np.sqrt(vh) + eps) + wd * w
    w1 = w - lr * upd
    tol = 2 * U32 * np.abs(w1) + 5e-4 * lr * (np.abs(mh / (np.sqrt(vh) + eps)) + wd * np.abs(w)) + 1e-12
    return w1, m1, v1, tol
