"""FP64 CPU oracle for FastMap's relative-translation grid search (arXiv 2505.04612).

TEST INFRASTRUCTURE ONLY.  The plain, slow, obviously correct reference the
HIP grid-search call is checked against.  Only the tests, the package's smoke
check and the benchmark's CPU-baseline leg may import it; the product path
never does.  It imports nothing from the package (only the epipolar oracle's
6D map) and computes in float64.

What it follows (appendix on global translation, "Relative Translation"):
after rotation averaging, the relative rotation of every pair is recomputed
from the global rotations, R_ij = R_j R_i^T, and the unit relative
translation is re-estimated by a search over candidate unit vectors: the
mean epipolar error of each candidate is evaluated and the lowest wins.

Readings where the paper is silent (each also listed in the design notes):
  G1  "mean epipolar error" is the mean over the pair's matches of the
      squared algebraic error (x2~^T [t]_x R_ij x1~)^2, evaluated from the
      pair's Gram W_n (App. B.6): e(t) = flatten([t]_x R_ij) is linear in t,
      e = B t, so the error is t^T (B^T W_n B) t / |Q_n|, a 3x3 form per pair;
  G2  the candidates are a set of unit vectors supplied by the caller (a
      Fibonacci lattice by default: near-uniform, a two-parameter family on
      the sphere); the lowest index wins among equal errors;
  G3  the error is even in t, so the winner keeps the sign of the pair's
      prior estimate t_prior (the decomposition's, which settles the sign by
      cheirality): the winner is negated when its dot product with t_prior
      is negative;
  G4  a pair without matches keeps its prior estimate.
"""
from __future__ import annotations

import numpy as np

from .ea import rot_from_6d


def skew(v: np.ndarray) -> np.ndarray:
    out = np.zeros(v.shape[:-1] + (3, 3))
    out[..., 0, 1], out[..., 0, 2] = -v[..., 2], v[..., 1]
    out[..., 1, 0], out[..., 1, 2] = v[..., 2], -v[..., 0]
    out[..., 2, 0], out[..., 2, 1] = -v[..., 1], v[..., 0]
    return out


def fibonacci_sphere(C: int) -> np.ndarray:
    """C near-uniform unit vectors (golden-angle spiral) [C,3]."""
    k = np.arange(C) + 0.5
    z = 1.0 - 2.0 * k / C
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = np.pi * (3.0 - np.sqrt(5.0)) * np.arange(C)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


def relative_rotations(theta: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """R_ij = R_j R_i^T [P,3,3] from parameters [N,>=6] (a1, a2, ...)."""
    theta = np.asarray(theta, dtype=np.float64)
    R = rot_from_6d(theta[:, 0:3], theta[:, 3:6])
    pairs = np.asarray(pairs)
    return R[pairs[:, 1]] @ np.swapaxes(R[pairs[:, 0]], -1, -2)


def translation_forms(W: np.ndarray, Rij: np.ndarray) -> np.ndarray:
    """A_n = B^T W_n B [P,3,3] with B[:, k] = flatten([e_k]_x R_ij) (row-major),
    so that flatten([t]_x R_ij)^T W_n flatten([t]_x R_ij) = t^T A_n t.
    W [P,9,9] full Grams."""
    P = Rij.shape[0]
    B = np.zeros((P, 9, 3))
    for k in range(3):
        ek = np.zeros(3)
        ek[k] = 1.0
        B[:, :, k] = (skew(ek)[None] @ Rij).reshape(P, 9)
    return np.swapaxes(B, -1, -2) @ W @ B


def candidate_errors(W: np.ndarray, counts: np.ndarray, Rij: np.ndarray, cand: np.ndarray) -> np.ndarray:
    """Mean squared algebraic epipolar error of every candidate for every
    pair [P,C] (reading G1), straight from the definition: e = flatten([t]_x R_ij)
    per candidate, e^T W_n e / |Q_n| (0 matches: 0)."""
    cand = np.asarray(cand, dtype=np.float64)
    E = skew(cand)[None] @ Rij[:, None]               # [P,C,3,3]
    e = E.reshape(Rij.shape[0], cand.shape[0], 9)
    q = np.einsum("pca,pab,pcb->pc", e, W, e)
    return q / np.maximum(np.asarray(counts, dtype=np.float64), 1.0)[:, None]


def grid_search(W: np.ndarray, counts: np.ndarray, Rij: np.ndarray, cand: np.ndarray, t_prior: np.ndarray):
    """Re-estimated unit relative translations [P,3] and the winning candidate
    index per pair [P] (readings G2-G4)."""
    err = candidate_errors(W, counts, Rij, cand)
    best = np.argmin(err, axis=1)                     # first minimum
    t = np.asarray(cand, dtype=np.float64)[best]
    flip = np.sum(t * t_prior, axis=1) < 0.0
    t[flip] = -t[flip]
    empty = np.asarray(counts) == 0
    t[empty] = t_prior[empty]
    best = np.where(empty, -1, best)
    return t, best, err
