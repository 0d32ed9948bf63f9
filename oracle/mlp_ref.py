"""Reference page-access predictor (numpy, float64).  TEST INFRASTRUCTURE
ONLY: it checks the GPU training and inference kernels and is never called
by the product path.

The paper does not define a predictor (it prefetches nothing; its decrypt-on-
fault path is the fallback here).  The network is this project's reading of
the learned-prefetch extension:
  input   the last C fault deltas of a client as vocabulary ids (C = 16);
  embed   E[V, D] (D = 64); the C embeddings are concatenated -> x[B, C*D];
  layer 1 z1 = x W1 + b1, h1 = relu(z1)           (W1: C*D x H, H = 256)
  layer 2 z2 = h1 W2 + b2, h2 = relu(z2)          (W2: H x H)
  output  logits = h2 W3 + b3                      (W3: H x V, V = 1024)
  loss    mean over the batch of softmax cross-entropy against the id of
          the next fault delta;
  update  Adam (lr, beta1, beta2, eps) on float32 master weights.
Storage points: the GPU keeps weights and the activations x, h1, h2 in
bfloat16 (round to nearest even) and accumulates in float32.  ``round_fn``
lets the reference apply the same rounding at the same points; with the
identity it is the exact float64 network that the finite-difference pins
check.
"""
from __future__ import annotations

import numpy as np

PARAMS = ("E", "W1", "b1", "W2", "b2", "W3", "b3")


def bf16_round(a: np.ndarray) -> np.ndarray:
    """float -> nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def identity(a):
    return a


def init_params(rng: np.random.Generator, vocab=1024, context=16, embed=64,
                hidden=256) -> dict:
    """Scaled normal initialisation (std 1/sqrt(fan_in)); zero biases."""
    d_in = context * embed
    return {
        "E": rng.normal(0, 1.0, (vocab, embed)),
        "W1": rng.normal(0, 1 / np.sqrt(d_in), (d_in, hidden)),
        "b1": np.zeros(hidden),
        "W2": rng.normal(0, 1 / np.sqrt(hidden), (hidden, hidden)),
        "b2": np.zeros(hidden),
        "W3": rng.normal(0, 1 / np.sqrt(hidden), (hidden, vocab)),
        "b3": np.zeros(vocab),
    }


def forward(p: dict, ids: np.ndarray, round_fn=identity):
    """Returns (logits, cache).  ids: (B, C) integers in [0, V)."""
    B, C = ids.shape
    x = round_fn(p["E"][ids].reshape(B, -1))
    z1 = x @ p["W1"] + p["b1"]
    h1 = round_fn(np.maximum(z1, 0.0))
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = round_fn(np.maximum(z2, 0.0))
    logits = h2 @ p["W3"] + p["b3"]
    return logits, {"ids": ids, "x": x, "z1": z1, "h1": h1, "z2": z2,
                    "h2": h2}


def loss_and_grads(p: dict, ids: np.ndarray, targets: np.ndarray,
                   round_fn=identity, grad_round_fn=identity):
    """Mean softmax cross-entropy and the gradient of every parameter.
    ``grad_round_fn`` rounds the gradient at the points where the GPU feeds
    a gradient into a bfloat16 matrix product (dlogits, dz2, dz1)."""
    logits, c = forward(p, ids, round_fn)
    B = ids.shape[0]
    m = logits.max(axis=1, keepdims=True)
    e = np.exp(logits - m)
    s = e.sum(axis=1, keepdims=True)
    logp = logits - m - np.log(s)
    loss = -logp[np.arange(B), targets].mean()
    dlogits = e / s
    dlogits[np.arange(B), targets] -= 1.0
    dlogits /= B
    dl = grad_round_fn(dlogits)
    g = {}
    g["W3"] = c["h2"].T @ dl
    g["b3"] = dlogits.sum(axis=0)
    dz2 = (dl @ p["W3"].T) * (c["h2"] > 0)
    dz2r = grad_round_fn(dz2)
    g["W2"] = c["h1"].T @ dz2r
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2r @ p["W2"].T) * (c["h1"] > 0)
    dz1r = grad_round_fn(dz1)
    g["W1"] = c["x"].T @ dz1r
    g["b1"] = dz1.sum(axis=0)
    dx = (dz1r @ p["W1"].T).reshape(B, ids.shape[1], -1)
    dE = np.zeros_like(p["E"])
    np.add.at(dE, ids, dx)
    g["E"] = dE
    return loss, g


def adam_step(p: dict, g: dict, m: dict, v: dict, t: int, lr=1e-3,
              beta1=0.9, beta2=0.999, eps=1e-8) -> None:
    """One Adam update in place (t counts from 1)."""
    for k in PARAMS:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] * g[k]
        mh = m[k] / (1 - beta1 ** t)
        vh = v[k] / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


def topk_ids(logits: np.ndarray, k: int, exclude: int | None = None):
    """Top-k ids per row by logit, ties to the lower id; `exclude` is never
    returned."""
    out = np.empty((logits.shape[0], k), dtype=np.int64)
    for b in range(logits.shape[0]):
        row = logits[b].astype(np.float64).copy()
        order = sorted(range(row.size), key=lambda i: (-row[i], i))
        if exclude is not None:
            order = [i for i in order if i != exclude]
        out[b] = order[:k]
    return out
