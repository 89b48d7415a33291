"""FP64 CPU oracle for FastMap's global rotation averaging (arXiv 2505.04612).

TEST INFRASTRUCTURE ONLY.  The plain, slow, obviously correct reference the
HIP rotation-averaging calls are checked against.  Only the tests, the
package's smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does.  It imports nothing from the package (only the 6D
map and the Adam step of the epipolar oracle) and computes in float64.

What it follows:
  * Sec. 3.3 "Global Rotation": world-to-camera rotations R_i, parameterised
    by the 6D representation, minimise
        L_R = (1/|P|) sum_(i,j) d(R_j, R^{i->j} R_i),
        d(A, B) = arccos((tr(A^T B) - 1) / 2)
    (eq. rotation-objective and the geodesic distance after it) with a
    first-order optimiser;
  * the appendix on rotation initialisation: the L2 objective
    sum ||R_j - R^{i->j} R_i||^2 split by columns; the first columns solve an
    unconstrained least-squares problem (a non-trivial minimiser, normalised
    per camera to unit length), the second columns the same problem plus a
    penalty (1/|I|) sum (c1_i . c2_i)^2 against the first columns with the
    pair term weighted 1/|P|, normalised, made orthogonal to the first
    column by Gram-Schmidt; the third column is c1 x c2.

Readings where the paper is silent (each also listed in the design notes):
  Q1  the arccos argument is clipped to [-1, 1]; where it is +-1 (distance 0
      or pi) the subgradient is taken as 0;
  Q2  "a non-trivial solution ... using techniques like SVD": the unit vector
      minimising the quadratic form, i.e. the eigenvector of the smallest
      eigenvalue of its 3N x 3N matrix (numpy.linalg.eigh); its sign and,
      with noise-free data, its position within the 3-dimensional null space
      are a global rotation of the result, which no comparison depends on;
  Q3  the optimiser is Adam on (a1, a2) with the learning rate decaying
      exponentially from lr0 to lr0*frac over the loop (as the epipolar
      oracle's reading R5);
  Q4  the pair-filtering step of the appendix (inlier-count thresholds) is
      upstream data preparation and not part of this stage.
"""
from __future__ import annotations

import numpy as np

from .ea import adam_step, rot_from_6d


# ------------------------------------------------------------------ objective

def geodesic(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """d(A, B) = arccos((tr(A^T B) - 1)/2) for stacks [...,3,3] (reading Q1)."""
    c = (np.einsum("...ab,...ab->...", A, B) - 1.0) / 2.0
    return np.arccos(np.clip(c, -1.0, 1.0))


def rotations(theta6: np.ndarray) -> np.ndarray:
    """R [N,3,3] from the 6D parameters [N,6] = (a1, a2)."""
    theta6 = np.asarray(theta6, dtype=np.float64)
    return rot_from_6d(theta6[:, 0:3], theta6[:, 3:6])


def loss(theta6: np.ndarray, pairs: np.ndarray, Rrel: np.ndarray) -> float:
    """L_R (eq. rotation-objective)."""
    P = len(pairs)
    if P == 0:
        return 0.0
    R = rotations(theta6)
    pairs = np.asarray(pairs)
    return float(geodesic(R[pairs[:, 1]], np.asarray(Rrel, np.float64) @ R[pairs[:, 0]]).sum() / P)


def gs_adjoint(theta6: np.ndarray, gR: np.ndarray) -> np.ndarray:
    """dL/d(a1, a2) [N,6] from dL/dR [N,3,3] through R = [b1 b2 b3]:
    b1 = a1/|a1|, u2 = a2 - (b1.a2) b1, b2 = u2/|u2|, b3 = b1 x b2."""
    a1, a2 = theta6[:, 0:3], theta6[:, 3:6]
    n1 = np.linalg.norm(a1, axis=-1, keepdims=True)
    b1 = a1 / n1
    d12 = np.sum(b1 * a2, axis=-1, keepdims=True)
    u2 = a2 - d12 * b1
    n2 = np.linalg.norm(u2, axis=-1, keepdims=True)
    b2 = u2 / n2
    g1, g2, g3 = gR[:, :, 0], gR[:, :, 1], gR[:, :, 2]
    # b3 = b1 x b2
    g1 = g1 + np.cross(b2, g3)
    g2 = g2 + np.cross(g3, b1)
    # b2 = u2/|u2|
    gu = (g2 - np.sum(b2 * g2, -1, keepdims=True) * b2) / n2
    # u2 = a2 - (b1.a2) b1
    ga2 = gu - b1 * np.sum(b1 * gu, -1, keepdims=True)
    g1 = g1 - d12 * gu - a2 * np.sum(b1 * gu, -1, keepdims=True)
    # b1 = a1/|a1|
    ga1 = (g1 - np.sum(b1 * g1, -1, keepdims=True) * b1) / n1
    return np.concatenate([ga1, ga2], axis=1)


def loss_grad(theta6: np.ndarray, pairs: np.ndarray, Rrel: np.ndarray):
    """(L_R, dL_R/dtheta [N,6]).  With c = (tr(R_j^T Q R_i) - 1)/2, Q = R^{i->j}:
    dd/dc = -1/sqrt(1 - c^2); dc/dR_j = Q R_i / 2; dc/dR_i = Q^T R_j / 2."""
    theta6 = np.asarray(theta6, dtype=np.float64)
    N, P = theta6.shape[0], len(pairs)
    if P == 0:
        return 0.0, np.zeros((N, 6))
    pairs = np.asarray(pairs)
    Q = np.asarray(Rrel, dtype=np.float64)
    R = rotations(theta6)
    i, j = pairs[:, 0], pairs[:, 1]
    QRi = Q @ R[i]
    c = (np.einsum("pab,pab->p", R[j], QRi) - 1.0) / 2.0
    L = float(np.arccos(np.clip(c, -1.0, 1.0)).sum() / P)
    inside = np.abs(c) < 1.0
    gc = np.zeros(P)
    gc[inside] = -1.0 / (P * np.sqrt(1.0 - c[inside] ** 2))
    gR = np.zeros((N, 3, 3))
    np.add.at(gR, j, 0.5 * gc[:, None, None] * QRi)
    np.add.at(gR, i, 0.5 * gc[:, None, None] * (np.swapaxes(Q, -1, -2) @ R[j]))
    return L, gs_adjoint(theta6, gR)


# ------------------------------------------------------------------ optimisation loop

def lr_at(lr0: float, frac: float, K: int, k: int) -> float:
    return lr0 * frac ** (k / K)


def solve(theta0: np.ndarray, pairs: np.ndarray, Rrel: np.ndarray, K: int, lr0: float = 1e-2,
          frac: float = 1e-2, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-12):
    """K Adam steps on L_R from theta0 [N,6]; returns (theta, loss trace [K])
    with L_R before each update."""
    th = np.array(theta0, dtype=np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    trace = np.zeros(K)
    for k in range(K):
        trace[k], g = loss_grad(th, pairs, Rrel)
        th, m, v = adam_step(th, g, m, v, k + 1, lr_at(lr0, frac, K, k), beta1, beta2, eps)
    return th, trace


# ------------------------------------------------------------------ initialisation (appendix)

def column_system(pairs: np.ndarray, Rrel: np.ndarray, N: int) -> np.ndarray:
    """The 3N x 3N matrix A of sum_(i,j) ||x_j - R^{i->j} x_i||^2 = x^T A x,
    x = (x_0, ..., x_{N-1}) stacked 3-vectors."""
    A = np.zeros((3 * N, 3 * N))
    I3 = np.eye(3)
    for (i, j), Q in zip(np.asarray(pairs), np.asarray(Rrel, dtype=np.float64)):
        si, sj = slice(3 * i, 3 * i + 3), slice(3 * j, 3 * j + 3)
        A[sj, sj] += I3
        A[si, si] += Q.T @ Q
        A[sj, si] -= Q
        A[si, sj] -= Q.T
    return A


def smallest_eigvec(A: np.ndarray) -> np.ndarray:
    w, V = np.linalg.eigh(A)
    return V[:, 0]


def _unit_rows(x: np.ndarray) -> np.ndarray:
    return x / np.linalg.norm(x, axis=1, keepdims=True)


def initialise(pairs: np.ndarray, Rrel: np.ndarray, N: int):
    """Rotations [N,3,3] from the column-wise least-squares problems of the
    appendix.  Returns (R, info) with the first and second column vectors
    before normalisation and the two matrices."""
    P = len(pairs)
    A = column_system(pairs, Rrel, N)
    x = smallest_eigvec(A).reshape(N, 3)
    c1 = _unit_rows(x)
    B = A / P
    for i in range(N):
        B[3 * i:3 * i + 3, 3 * i:3 * i + 3] += np.outer(c1[i], c1[i]) / N
    y = smallest_eigvec(B).reshape(N, 3)
    c2 = _unit_rows(y)
    c2 = _unit_rows(c2 - np.sum(c1 * c2, axis=1, keepdims=True) * c1)
    c3 = np.cross(c1, c2)
    R = np.stack([c1, c2, c3], axis=-1)
    return R, {"x": x, "y": y, "A": A, "B": B}


def relative_rotation_errors(Ra: np.ndarray, Rb: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """Per pair, the angle (degrees) between the relative rotations R_j R_i^T
    of two solutions (independent of a global rotation of either)."""
    pairs = np.asarray(pairs)
    i, j = pairs[:, 0], pairs[:, 1]
    Qa = Ra[j] @ np.swapaxes(Ra[i], -1, -2)
    Qb = Rb[j] @ np.swapaxes(Rb[i], -1, -2)
    return np.degrees(geodesic(Qa, Qb))
