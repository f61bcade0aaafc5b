"""Learned pivot proposer for the cross (not part of the paper's method).

Oracle (test infrastructure only).

The cross of Section 3.3 chooses column pivots J by alternating maxvol sweeps, started from
the same call site's pivots of the previous step.  The proposer replaces the sweeps by a
score per column index: a multilayer perceptron maps 16 features of index j to a logit, the
top-K indices become J, and one refinement sweep follows.  This module holds the plain
float64 definitions the GPU kernels are checked against:

  features   the 16 features of every column index j of an n2-column cross, computed from
             the second core B0 (n2 x r) of the cross's starting TT and the previous pivots:
               0      1 if j is a previous pivot
               1      exp(-d / 2), d = distance from j to the nearest previous pivot
               2..6   log(1 + lev(j + o)),  o = -2..2, lev(j) = n2 |B0[j]|^2 / |B0|_F^2
               7..11  log(1 + jump(j + o)), o = -2..2,
                      jump(j) = n2 |B0[j + 1] - B0[j]|^2 / |B0|_F^2 (0 at the last row)
               12     j / n2
               13,14  sin, cos of 2 pi j / n2
               15     1
             indices j + o outside [0, n2) are clamped to the range.
  forward    h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), s = h2 w3 + b3
             (16 -> 256 -> 256 -> 1)
  loss       weighted logistic loss  L = sum_i w_i (log(1 + e^{s_i}) - y_i s_i) / N with
             w_i = pos_weight for pivots (y_i = 1) and 1 otherwise
  backward   gradients of L by the chain rule, written out layer by layer
  adam       one Adam step (Kingma and Ba 2015)
"""
from __future__ import annotations

import math
from typing import Dict, Sequence

import numpy as np

F = 16
H = 256


def features(B0: np.ndarray, J_prev: Sequence[int]) -> np.ndarray:
    n2 = B0.shape[0]
    nrm2 = float(np.sum(B0 * B0))
    if nrm2 <= 0.0:
        nrm2 = 1.0
    lev = n2 * np.sum(B0 * B0, axis=1) / nrm2
    nxt = np.minimum(np.arange(n2) + 1, n2 - 1)
    dB = B0[nxt] - B0
    jump = n2 * np.sum(dB * dB, axis=1) / nrm2
    X = np.zeros((n2, F))
    J = np.asarray(sorted(set(int(j) for j in J_prev)), dtype=np.int64)
    idx = np.arange(n2)
    if J.size:
        X[J, 0] = 1.0
        d = np.min(np.abs(idx[:, None] - J[None, :]), axis=1)
    else:
        d = np.full(n2, float(n2))
    X[:, 1] = np.exp(-d / 2.0)
    for k, o in enumerate(range(-2, 3)):
        jj = np.clip(idx + o, 0, n2 - 1)
        X[:, 2 + k] = np.log1p(lev[jj])
        X[:, 7 + k] = np.log1p(jump[jj])
    X[:, 12] = idx / n2
    X[:, 13] = np.sin(2.0 * math.pi * idx / n2)
    X[:, 14] = np.cos(2.0 * math.pi * idx / n2)
    X[:, 15] = 1.0
    return X


def init_weights(rng: np.random.Generator) -> Dict[str, np.ndarray]:
    """He-normal weights, zero biases."""
    return {"W1": rng.standard_normal((F, H)) * math.sqrt(2.0 / F), "b1": np.zeros(H),
            "W2": rng.standard_normal((H, H)) * math.sqrt(2.0 / H), "b2": np.zeros(H),
            "w3": rng.standard_normal(H) * math.sqrt(1.0 / H), "b3": np.zeros(1)}


def forward(p: Dict[str, np.ndarray], X: np.ndarray):
    z1 = X @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    s = h2 @ p["w3"] + p["b3"][0]
    return s, (X, h1, h2)


def loss(s: np.ndarray, y: np.ndarray, pos_weight: float) -> float:
    w = np.where(y > 0.5, pos_weight, 1.0)
    sp = np.logaddexp(0.0, s)            # log(1 + e^s), stable
    return float(np.sum(w * (sp - y * s)) / s.size)


def backward(p: Dict[str, np.ndarray], cache, s: np.ndarray, y: np.ndarray,
             pos_weight: float) -> Dict[str, np.ndarray]:
    X, h1, h2 = cache
    N = s.size
    w = np.where(y > 0.5, pos_weight, 1.0)
    sig = 1.0 / (1.0 + np.exp(-s))
    ds = w * (sig - y) / N                 # dL/ds
    g = {"w3": h2.T @ ds, "b3": np.array([ds.sum()])}
    dh2 = np.outer(ds, p["w3"]) * (h2 > 0.0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ p["W2"].T) * (h1 > 0.0)
    g["W1"] = X.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return g


def adam_step(p, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """In-place Adam update of p (m, v: first and second moment dicts; t >= 1)."""
    for k in p:
        m[k] = b1 * m[k] + (1.0 - b1) * g[k]
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k]
        mh = m[k] / (1.0 - b1 ** t)
        vh = v[k] / (1.0 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
