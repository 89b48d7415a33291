"""FP64 CPU oracle for focal-length refinement inside epipolar adjustment
(FastMap, arXiv 2505.04612).

TEST INFRASTRUCTURE ONLY.  The plain, slow, obviously correct reference the
HIP focal-refinement call is checked against.  Only the tests, the package's
smoke check and the benchmark's CPU-baseline leg may import it; the product
path never does.  It imports nothing from the package (only the epipolar
oracle's pose helpers and Adam) and computes in float64.

What it follows: Sec. 3.3, the sentence after the IRLS paragraph - the focal
lengths can be optimised together with the poses by building them into the
essential matrices, which then are fundamental matrices.  With coordinates
normalised by a focal estimate f0_i per camera, x~ = K0^-1 x_pixel, and a
refined focal f_i = sigma_i f0_i, the camera ray is S_i x~ with
S_i = diag(1/sigma_i, 1/sigma_i, 1), so the pair's matrix acting on the
stored coordinates is F_n = S_j E_n S_i.

Readings where the paper is silent (each also listed in the design notes):
  F1  each pair's term is normalised by |F_n|_F^2: L = (1/Z) sum_n
      f_n^T W_n f_n / f_n^T f_n, f_n = flatten(F_n) row-major.  Without it,
      growing sigma shrinks F and lowers the algebraic loss toward zero (for
      small relative rotations E_22 ~ 0), a trivial minimum; with unit t_hat,
      |E|_F^2 = 2, so at sigma = 1 the loss is exactly half the epipolar one;
  F2  one focal per camera, parameterised by phi_i = log sigma_i (positive
      focal lengths);
  F3  everything else (E_n, unit relative translation, 6D rotations, Z,
      Adam) as in the epipolar oracle.
"""
from __future__ import annotations

import numpy as np

from .ea import adam_step, skew


def _scales(phi: np.ndarray) -> np.ndarray:
    """s_i = (1/sigma_i, 1/sigma_i, 1) [N,3]."""
    e = np.exp(-np.asarray(phi, dtype=np.float64))
    return np.stack([e, e, np.ones_like(e)], axis=1)


def fundamentals(theta: np.ndarray, phi: np.ndarray, pairs: np.ndarray):
    """(F [P,3,3], E [P,3,3]) with F_n = S_j E_n S_i."""
    from .ea import essentials
    E = essentials(theta, pairs)
    s = _scales(phi)
    pairs = np.asarray(pairs)
    F = s[pairs[:, 1]][:, :, None] * E * s[pairs[:, 0]][:, None, :]
    return F, E


def loss(theta: np.ndarray, phi: np.ndarray, pairs: np.ndarray, W: np.ndarray, inv_Z: float) -> float:
    """L = inv_Z * sum_n f^T W f / f^T f (reading F1).  W [P,9,9]."""
    F, _ = fundamentals(theta, phi, pairs)
    f = F.reshape(-1, 9)
    num = np.einsum("pa,pab,pb->p", f, W, f)
    den = np.sum(f * f, axis=1)
    return float(inv_Z * np.sum(np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)))


def loss_grad(theta: np.ndarray, phi: np.ndarray, pairs: np.ndarray, W: np.ndarray, inv_Z: float):
    """(L, dL/dtheta [N,9], dL/dphi [N]).  dL/df = 2 inv_Z (W f - q f)/(f^T f),
    q = f^T W f / f^T f; dF/dE through the scales; dF_ab/dphi_j = -F_ab for
    a < 2, dF_ab/dphi_i = -F_ab for b < 2; then the epipolar chain rule
    through E = [t_hat]_x R_ij, the normalisation of t_ij, R_ij = R_j R_i^T
    and the Gram-Schmidt map."""
    theta = np.asarray(theta, dtype=np.float64)
    N = theta.shape[0]
    pairs = np.asarray(pairs)
    i, j = pairs[:, 0], pairs[:, 1]
    a1, a2, t = theta[:, 0:3], theta[:, 3:6], theta[:, 6:9]
    n1 = np.linalg.norm(a1, axis=-1, keepdims=True)
    b1 = a1 / n1
    d12 = np.sum(b1 * a2, axis=-1, keepdims=True)
    u2 = a2 - d12 * b1
    n2 = np.linalg.norm(u2, axis=-1, keepdims=True)
    b2 = u2 / n2
    b3 = np.cross(b1, b2)
    R = np.stack([b1, b2, b3], axis=-1)
    Rij = R[j] @ np.swapaxes(R[i], -1, -2)
    sv = t[j] - np.einsum("pab,pb->pa", Rij, t[i])
    ns = np.linalg.norm(sv, axis=-1, keepdims=True)
    live = ns[:, 0] > 0
    th = sv / np.where(ns > 0, ns, 1.0)
    T = skew(th)
    E = T @ Rij
    s = _scales(phi)
    M = s[j][:, :, None] * s[i][:, None, :]          # F = M * E elementwise
    F = M * E
    f = F.reshape(-1, 9)
    Wf = np.einsum("pab,pb->pa", W, f)
    den = np.sum(f * f, axis=1)
    den_safe = np.where(live, den, 1.0)
    q = np.where(live, np.sum(f * Wf, axis=1) / den_safe, 0.0)
    L = float(inv_Z * np.sum(q))
    GF = (2.0 * inv_Z * (Wf - q[:, None] * f) / den_safe[:, None]).reshape(-1, 3, 3)
    GF[~live] = 0.0
    GE = GF * M
    gphi = np.zeros(N)
    GFF = GF * F
    np.add.at(gphi, j, -GFF[:, 0:2, :].sum(axis=(1, 2)))
    np.add.at(gphi, i, -GFF[:, :, 0:2].sum(axis=(1, 2)))
    # epipolar chain rule from dL/dE
    A = GE @ np.swapaxes(Rij, -1, -2)
    dRij = np.swapaxes(T, -1, -2) @ GE
    gth = np.stack([A[:, 2, 1] - A[:, 1, 2], A[:, 0, 2] - A[:, 2, 0], A[:, 1, 0] - A[:, 0, 1]], -1)
    gs = (gth - np.sum(th * gth, -1, keepdims=True) * th) / np.where(ns > 0, ns, 1.0)
    gs[~live] = 0.0
    dRij = dRij - gs[:, :, None] * t[i][:, None, :]
    gt = np.zeros((N, 3))
    np.add.at(gt, j, gs)
    np.add.at(gt, i, -np.einsum("pba,pb->pa", Rij, gs))
    gR = np.zeros((N, 3, 3))
    np.add.at(gR, j, dRij @ R[i])
    np.add.at(gR, i, np.swapaxes(dRij, -1, -2) @ R[j])
    g1, g2, g3 = gR[:, :, 0], gR[:, :, 1], gR[:, :, 2]
    g1 = g1 + np.cross(b2, g3)
    g2 = g2 + np.cross(g3, b1)
    gu = (g2 - np.sum(b2 * g2, -1, keepdims=True) * b2) / n2
    ga2 = gu - b1 * np.sum(b1 * gu, -1, keepdims=True)
    g1 = g1 - d12 * gu - a2 * np.sum(b1 * gu, -1, keepdims=True)
    ga1 = (g1 - np.sum(b1 * g1, -1, keepdims=True) * b1) / n1
    return L, np.concatenate([ga1, ga2, gt], axis=1), gphi


def solve(theta0, phi0, pairs, W, inv_Z, K: int, lr_rot=3e-3, lr_t=1e-2, lr_phi=1e-2, frac=1e-2,
          beta1=0.9, beta2=0.999, eps=1e-12):
    """K Adam steps on (theta, phi) with exponentially decaying rates;
    returns (theta, phi, loss trace [K])."""
    th = np.array(theta0, dtype=np.float64)
    ph = np.array(phi0, dtype=np.float64)
    m, v = np.zeros_like(th), np.zeros_like(th)
    mp, vp = np.zeros_like(ph), np.zeros_like(ph)
    lr0 = np.array([lr_rot] * 6 + [lr_t] * 3)
    trace = np.zeros(K)
    for k in range(K):
        trace[k], g, gp = loss_grad(th, ph, pairs, W, inv_Z)
        f = frac ** (k / K)
        th, m, v = adam_step(th, g, m, v, k + 1, lr0 * f, beta1, beta2, eps)
        ph, mp, vp = adam_step(ph, gp, mp, vp, k + 1, lr_phi * f, beta1, beta2, eps)
    return th, ph, trace
