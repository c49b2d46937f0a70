"""Oracle: FP64 surrogate network of the log-cycle estimate (not in the paper).

Test infrastructure only (see the package docstring); never imported by the product path.

Network (one network shared by all kernels, conditioned on a learned scalar embedding e_k
per kernel):
    x  = (log2 N / 26, log2 bx / 10, log2 by / 10, e_k)
    h1 = relu(W1 x + b1)            W1: [H1][4]
    h2 = relu(W2 h1 + b2)           W2: [H2][H1]
    y  = w3 . h2 + b3               prediction of the standardised log-cycles (ln C - mu) / sigma
Loss: mean over the batch of (y - t)^2.  Optimiser: Adam with bias correction,
    m = b1 m + (1 - b1) g;  v = b2 v + (1 - b2) g^2;  p -= lr * (m / (1 - b1^s)) / (sqrt(v / (1 - b2^s)) + eps)
where s is the 1-based step count.
"""
from __future__ import annotations

import numpy as np

PARAM_NAMES = ("W1", "b1", "W2", "b2", "w3", "b3", "emb")


def features(N, bx, by, emb_k):
    N, bx, by = (np.asarray(a, np.float64) for a in (N, bx, by))
    return np.stack([np.log2(N) / 26.0, np.log2(bx) / 10.0, np.log2(by) / 10.0,
                     np.asarray(emb_k, np.float64)], axis=1)


def forward(p, kid, N, bx, by):
    """Returns (y [B], cache) in FP64."""
    x = features(N, bx, by, p["emb"][np.asarray(kid)])
    a1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ p["w3"] + p["b3"]
    return y, {"x": x, "a1": a1, "h1": h1, "a2": a2, "h2": h2, "kid": np.asarray(kid)}


def bf16_round(a):
    """Round to the nearest bfloat16 value (8 significand bits, ties to even), from the value's
    FP32 rounding; returned as FP64.  bfloat16 is FP32 with the low 16 bits of the encoding
    dropped, so rounding adds half of the dropped range (minus one unless the kept part is odd)
    and clears the low half-word."""
    b = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def forward_bf16(p, kid, N, bx, by):
    """The forward pass with the 256 x 256 layer's operands in bfloat16, as the selection kernel
    takes them: W2 and the first hidden layer h1 rounded to bfloat16 (from FP32), every other
    step in FP64.  Returns y [B]."""
    x = features(N, bx, by, p["emb"][np.asarray(kid)])
    h1 = bf16_round(np.maximum(x @ p["W1"].T + p["b1"], 0.0))
    h2 = np.maximum(h1 @ bf16_round(p["W2"]).T + p["b2"], 0.0)
    return h2 @ p["w3"] + p["b3"]


def loss_and_grads(p, kid, N, bx, by, t):
    """MSE loss and its analytic gradient with respect to every parameter (FP64)."""
    y, c = forward(p, kid, N, bx, by)
    B = y.shape[0]
    r = y - np.asarray(t, np.float64)
    loss = float(np.mean(r * r))
    dy = 2.0 * r / B
    g = {}
    g["w3"] = c["h2"].T @ dy
    g["b3"] = np.array(dy.sum())
    da2 = np.outer(dy, p["w3"]) * (c["a2"] > 0)
    g["W2"] = da2.T @ c["h1"]
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ p["W2"]) * (c["a1"] > 0)
    g["W1"] = da1.T @ c["x"]
    g["b1"] = da1.sum(axis=0)
    dx3 = da1 @ p["W1"][:, 3]
    g["emb"] = np.zeros_like(p["emb"])
    np.add.at(g["emb"], c["kid"], dx3)
    return loss, g


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of every parameter; step is 1-based.  Returns new (p, m, v)."""
    p2, m2, v2 = {}, {}, {}
    for k in PARAM_NAMES:
        m2[k] = beta1 * m[k] + (1.0 - beta1) * g[k]
        v2[k] = beta2 * v[k] + (1.0 - beta2) * g[k] * g[k]
        mh = m2[k] / (1.0 - beta1 ** step)
        vh = v2[k] / (1.0 - beta2 ** step)
        p2[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p2, m2, v2


def zeros_like(p):
    return {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in p.items()}
