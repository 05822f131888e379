"""Oracle of the learned proposal's network: a 16-256-256-1 perceptron with
ReLU and a sigmoid output, trained with binary cross-entropy and Adam.

Test infrastructure: FP64 NumPy.  The learned proposal is not part of the
paper (which only cites learned indexers as prior art, Sec. 2); this module
fixes what the GPU network computes so that it can be checked.

Precision contract shared with the GPU: weights and the activations that enter
a product are rounded to bfloat16 (round to nearest even) first; products and
sums are exact here (FP64) and FP32-accumulated on the GPU.
  forward:  xb = bf16(x); a1 = xb W1b^T + b1; h1b = bf16(relu(a1));
            a2 = h1b W2b^T + b2; h2b = bf16(relu(a2)); z = h2b . w3b + b3;
            p = sigmoid(z)
  backward (loss = mean BCE over the batch):
            dz = (p - y) / B; dw3 = sum dz h2b; db3 = sum dz;
            dh2 = dz w3b [a2 > 0]; dW2 = bf16(dh2)^T h1b; db2 = sum dh2;
            dh1 = (bf16(dh2) W2b) [a1 > 0]; dW1 = bf16(dh1)^T xb; db1 = sum dh1
  Adam:     m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
            w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)   (FP32 masters)
With round=False every bfloat16 rounding is skipped (used for the
finite-difference pins).
"""
from __future__ import annotations

import numpy as np


def bf16(x):
    """Round to bfloat16, nearest even, returned as FP64 (exact)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def init(n_in=16, n_hidden=256, seed=0):
    """He-uniform weights, zero biases (FP64 masters, stored as FP32 values)."""
    rng = np.random.default_rng(seed)
    lim1 = np.sqrt(6.0 / n_in)
    lim2 = np.sqrt(6.0 / n_hidden)
    p = {"W1": rng.uniform(-lim1, lim1, (n_hidden, n_in)),
         "b1": np.zeros(n_hidden),
         "W2": rng.uniform(-lim2, lim2, (n_hidden, n_hidden)),
         "b2": np.zeros(n_hidden),
         "w3": rng.uniform(-lim2, lim2, n_hidden) * 0.1,
         "b3": np.zeros(1)}
    return {k: v.astype(np.float32).astype(np.float64) for k, v in p.items()}


def _r(x, round_):
    return bf16(x) if round_ else np.asarray(x, dtype=np.float64)


def forward(p, x, round_=True):
    xb = _r(x, round_)
    a1 = xb @ _r(p["W1"], round_).T + p["b1"]
    h1 = _r(np.maximum(a1, 0.0), round_)
    a2 = h1 @ _r(p["W2"], round_).T + p["b2"]
    h2 = _r(np.maximum(a2, 0.0), round_)
    z = h2 @ _r(p["w3"], round_) + p["b3"][0]
    prob = 1.0 / (1.0 + np.exp(-z))
    return prob, {"xb": xb, "a1": a1, "h1": h1, "a2": a2, "h2": h2, "z": z}


def loss(p, x, y, round_=True):
    prob, c = forward(p, x, round_)
    z = c["z"]
    # stable BCE with logits
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def backward(p, x, y, round_=True):
    prob, c = forward(p, x, round_)
    B = x.shape[0]
    dz = (prob - y) / B
    g = {"w3": c["h2"].T @ dz, "b3": np.array([dz.sum()])}
    dh2 = np.outer(dz, _r(p["w3"], round_)) * (c["a2"] > 0)
    dh2b = _r(dh2, round_)
    g["W2"] = dh2b.T @ c["h1"]
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2b @ _r(p["W2"], round_)) * (c["a1"] > 0)
    dh1b = _r(dh1, round_)
    g["W1"] = dh1b.T @ c["xb"]
    g["b1"] = dh1.sum(axis=0)
    return g, prob


def adam(p, g, state, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step on the masters (t counts from 1).  Returns new (p, state)."""
    np_, ns = {}, {}
    for k in p:
        m = b1 * state.get(("m", k), 0.0) + (1 - b1) * g[k]
        v = b2 * state.get(("v", k), 0.0) + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        np_[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
        ns[("m", k)] = m
        ns[("v", k)] = v
    return np_, ns
