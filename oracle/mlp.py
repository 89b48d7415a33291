"""FP64 CPU oracle of the learned-weight form (test infrastructure only).

A per-match robust weight is proposed by a small MLP from three features of
the match at the current poses (the paper weights matches by IRLS, Sec. 3.3;
the learned proposal is not part of the paper, so nothing here is pinned
by a printed value of the paper: the pins are finite differences and closed
forms):
  f0 = log max(|r|, delta), r = x2~^T E_n x1~ the epipolar residual;
  f1 = log |Q_n|, the number of matches of the pair;
  f2 = parallax angle between the bearing rays R_i^T x1~ and R_j^T x2~ (rad).
Network: standardise (f - mean) / std, then 3 -> 64 -> 64 -> 1 with ReLU,
ReLU, sigmoid.  Weights are row-major [out, in].
"""
from __future__ import annotations

import numpy as np

from . import ea

SHAPES = {"W1": (64, 3), "b1": (64,), "W2": (64, 64), "b2": (64,), "W3": (1, 64), "b3": (1,)}


def features(theta, pairs, offsets, uv, delta):
    r = ea.residuals(theta, pairs, offsets, uv)
    counts = np.diff(np.asarray(offsets, dtype=np.int64))
    f0 = np.log(np.maximum(np.abs(r), delta))
    f1 = np.repeat(np.log(np.maximum(counts, 1).astype(np.float64)), counts)
    R, _ = ea.poses_from_params(theta)
    x1, x2 = ea.homogeneous(uv)
    Ri = np.repeat(R[pairs[:, 0]], counts, axis=0)
    Rj = np.repeat(R[pairs[:, 1]], counts, axis=0)
    a = np.einsum("mba,mb->ma", Ri, x1)      # R_i^T x1~
    b = np.einsum("mba,mb->ma", Rj, x2)      # R_j^T x2~
    f2 = np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.sum(a * b, axis=1))
    return np.stack([f0, f1, f2], axis=1)


def init_params(seed=0):
    rng = np.random.default_rng(seed)
    p = {}
    for k, s in SHAPES.items():
        if k.startswith("W"):
            p[k] = rng.normal(0.0, np.sqrt(2.0 / s[1]), size=s)
        else:
            p[k] = np.zeros(s)
    return p


def forward(p, feats, mean, std):
    x = (np.asarray(feats, dtype=np.float64) - mean) / std
    z1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ p["W3"].T + p["b3"]
    out = 1.0 / (1.0 + np.exp(-z3[:, 0]))
    return out, (x, z1, h1, z2, h2)


def backward(p, feats, mean, std, dout):
    """Gradients of sum_m dout[m] * out[m] with respect to every weight."""
    out, (x, z1, h1, z2, h2) = forward(p, feats, mean, std)
    d3 = np.asarray(dout, dtype=np.float64) * out * (1.0 - out)
    g = {"W3": d3[None, :] @ h2, "b3": np.array([d3.sum()])}
    dh2 = d3[:, None] * p["W3"][0][None, :] * (z2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ p["W2"]) * (z1 > 0)
    g["W1"] = dh1.T @ x
    g["b1"] = dh1.sum(axis=0)
    return g
