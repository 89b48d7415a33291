"""FP64 CPU oracle for FastMap's epipolar adjustment (arXiv 2505.04612).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
reference the HIP library is checked against.  Only the tests, the package's
smoke check and the benchmark's CPU-baseline leg may import it; the product
path never does.  It shares no code with the HIP path (it imports nothing from
the package) and computes everything in float64 with NumPy.

What it follows (all in Sec. 3.3 "Epipolar Adjustment" and App. B.6):
  * the robust objective, eq. (epipolar-objective): mean over all point pairs
    of |x2~^T E_n x1~|;
  * its L2 form, eq. (epipolar-objective-l2), reorganised per image pair as a
    quadratic form e_n^T W_n e_n with W_n = sum_m w_nm w_nm^T and
    w_nm = flatten(x2~ x1~^T) (App. B.6);
  * IRLS: weights 1/|eps_hat| at the current poses, a weighted Gram, another
    optimisation loop, and a decaying outlier-filter threshold (the paragraph
    after the IRLS equation);
  * an adaptive first-order optimiser (Adam, cited in Sec. 3.2);
  * the 6D rotation parameterisation with Gram-Schmidt (Sec. 3.3 "Global
    Rotation", which states it for the rotation stage).

Readings where the paper is silent or garbled (each also listed in the design
notes of the repository):
  R1  no factor 2: sum_m (w^T e)^2 = e^T W e exactly; the "2/Z" printed in
      eq. (epipolar-objective-l2) and App. B.6 does not follow from the
      derivation's own previous step.  L = (1/Z) sum_n e_n^T W_n e_n.
  R2  the App. B.6 "element-wise product" is a Frobenius inner product, and
      flatten is row-major: w[3a+b] = x2~[a] x1~[b], e[3a+b] = E[a,b].
  R3  E_n = [t_hat]_x R_ij with R_ij = R_j R_i^T, t_ij = t_j - R_ij t_i and
      t_hat = t_ij / |t_ij| (unit relative translation, which removes the
      trivial t -> 0 minimum of the epipolar objective).
  R4  rotations use the 6D representation (a1, a2) -> Gram-Schmidt columns.
  R5  Adam (beta 0.9/0.999, eps 1e-12), step counter from 1 in every
      optimisation loop (Adam state is reset when the weights change); the
      learning rate decays exponentially from lr0 to lr0*frac over the solve.
  R6  IRLS weight 1/max(|r|, delta), delta = 1e-4; matches with |r| > tau_k are
      filtered (weight 0); tau_0 = 0.1, tau_{k+1} = max(tau_k / 2, 0.01).
  R7  Z = number of matches with nonzero weight.
  R8  the first loop's weights are computed at the initial poses, as the paper
      does (it assumes a good initialisation); a flag switches the first loop
      to unit weights.
"""
from __future__ import annotations

import dataclasses

import numpy as np


# ------------------------------------------------------------------ inputs

def homogeneous(uv: np.ndarray):
    """Split [M,4] (u1, v1, u2, v2) into homogeneous x1~, x2~ [M,3] float64."""
    uv = np.asarray(uv, dtype=np.float64)
    one = np.ones((uv.shape[0], 1))
    return np.hstack([uv[:, 0:2], one]), np.hstack([uv[:, 2:4], one])


# ------------------------------------------------------------------ Gram (App. B.6)

def match_vectors(uv: np.ndarray) -> np.ndarray:
    """w_nm = flatten(x2~ x1~^T) (row-major), one 9-vector per match [M,9]."""
    x1, x2 = homogeneous(uv)
    return (x2[:, :, None] * x1[:, None, :]).reshape(-1, 9)


def pair_grams(uv: np.ndarray, offsets: np.ndarray, weights: np.ndarray | None = None) -> np.ndarray:
    """W_n = sum_m omega_m w_nm w_nm^T for every pair n, [P,9,9] float64.

    App. B.6 defines W_n as the sum of outer products of the per-match
    9-vectors; IRLS (Sec. 3.3) weights each term.  A pair without matches gets
    W_n = 0.
    """
    offsets = np.asarray(offsets, dtype=np.int64)
    P = offsets.size - 1
    out = np.zeros((P, 9, 9))
    for n in range(P):
        lo, hi = int(offsets[n]), int(offsets[n + 1])
        if hi == lo:
            continue
        w = match_vectors(uv[lo:hi])
        if weights is not None:
            om = np.asarray(weights[lo:hi], dtype=np.float64)
            out[n] = (w * om[:, None]).T @ w
        else:
            out[n] = w.T @ w
    return out


# ------------------------------------------------------------------ poses

def rot_from_6d(a1: np.ndarray, a2: np.ndarray) -> np.ndarray:
    """Gram-Schmidt of two 3-vectors into the columns of a rotation [N,3,3]:
    b1 = a1/|a1|, b2 = normalise(a2 - (b1.a2) b1), b3 = b1 x b2."""
    b1 = a1 / np.linalg.norm(a1, axis=-1, keepdims=True)
    u2 = a2 - np.sum(b1 * a2, axis=-1, keepdims=True) * b1
    b2 = u2 / np.linalg.norm(u2, axis=-1, keepdims=True)
    b3 = np.cross(b1, b2)
    return np.stack([b1, b2, b3], axis=-1)


def params_from_poses(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    """theta_i = (a1, a2, t) with a1, a2 the first two columns of R_i: [N,9]."""
    return np.concatenate([R[:, :, 0], R[:, :, 1], t], axis=1).astype(np.float64)


def poses_from_params(theta: np.ndarray):
    theta = np.asarray(theta, dtype=np.float64)
    return rot_from_6d(theta[:, 0:3], theta[:, 3:6]), theta[:, 6:9].copy()


def skew(v: np.ndarray) -> np.ndarray:
    """[v]_x such that [v]_x y = v x y, batched."""
    z = np.zeros(v.shape[:-1])
    return np.stack([
        np.stack([z, -v[..., 2], v[..., 1]], -1),
        np.stack([v[..., 2], z, -v[..., 0]], -1),
        np.stack([-v[..., 1], v[..., 0], z], -1)], -2)


def relative(R: np.ndarray, t: np.ndarray, pairs: np.ndarray):
    """R_ij = R_j R_i^T and t_ij = t_j - R_ij t_i for pairs (i, j)."""
    i, j = pairs[:, 0], pairs[:, 1]
    Rij = R[j] @ np.swapaxes(R[i], -1, -2)
    tij = t[j] - np.einsum("pab,pb->pa", Rij, t[i])
    return Rij, tij


def essentials(theta: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """E_n = [t_hat]_x R_ij per pair from the global poses [P,3,3] (reading R3)."""
    R, t = poses_from_params(theta)
    Rij, tij = relative(R, t, pairs)
    th = tij / np.linalg.norm(tij, axis=-1, keepdims=True)
    return skew(th) @ Rij


# ------------------------------------------------------------------ loss and gradient

def loss_from_grams(theta: np.ndarray, pairs: np.ndarray, W: np.ndarray, inv_Z: float) -> float:
    """L = inv_Z * sum_n e_n^T W_n e_n, eq. (epipolar-objective-l2) under R1."""
    e = essentials(theta, pairs).reshape(-1, 9)
    return float(inv_Z * np.einsum("pa,pab,pb->", e, W, e))


def pair_losses(theta, pairs, W):
    e = essentials(theta, pairs).reshape(-1, 9)
    return np.einsum("pa,pab,pb->p", e, W, e)


def loss_grad(theta: np.ndarray, pairs: np.ndarray, W: np.ndarray, inv_Z: float):
    """Loss and its analytic gradient with respect to theta [N,9].

    Chain rule through e^T W e, E = T R_ij with T = [t_hat]_x, the
    normalisation of t_ij, t_ij = t_j - R_ij t_i, R_ij = R_j R_i^T, and the
    Gram-Schmidt map from (a1, a2) to R.
    """
    theta = np.asarray(theta, dtype=np.float64)
    N = theta.shape[0]
    a1, a2, t = theta[:, 0:3], theta[:, 3:6], theta[:, 6:9]
    # forward
    n1 = np.linalg.norm(a1, axis=-1, keepdims=True)
    b1 = a1 / n1
    d12 = np.sum(b1 * a2, axis=-1, keepdims=True)
    u2 = a2 - d12 * b1
    n2 = np.linalg.norm(u2, axis=-1, keepdims=True)
    b2 = u2 / n2
    b3 = np.cross(b1, b2)
    R = np.stack([b1, b2, b3], axis=-1)
    i, j = pairs[:, 0], pairs[:, 1]
    Rij = R[j] @ np.swapaxes(R[i], -1, -2)
    s = t[j] - np.einsum("pab,pb->pa", Rij, t[i])
    ns = np.linalg.norm(s, axis=-1, keepdims=True)
    th = s / ns
    T = skew(th)
    E = T @ Rij
    e = E.reshape(-1, 9)
    We = np.einsum("pab,pb->pa", W, e)
    L = float(inv_Z * np.sum(e * We))
    # backward
    G = (2.0 * inv_Z * We).reshape(-1, 3, 3)            # dL/dE
    A = G @ np.swapaxes(Rij, -1, -2)                     # dL/dT
    dRij = np.swapaxes(T, -1, -2) @ G                    # dL/dR_ij via E
    gth = np.stack([A[:, 2, 1] - A[:, 1, 2], A[:, 0, 2] - A[:, 2, 0], A[:, 1, 0] - A[:, 0, 1]], -1)
    gs = (gth - np.sum(th * gth, -1, keepdims=True) * th) / ns
    dRij = dRij - gs[:, :, None] * t[i][:, None, :]
    gt = np.zeros((N, 3))
    np.add.at(gt, j, gs)
    np.add.at(gt, i, -np.einsum("pba,pb->pa", Rij, gs))
    gR = np.zeros((N, 3, 3))
    np.add.at(gR, j, dRij @ R[i])
    np.add.at(gR, i, np.swapaxes(dRij, -1, -2) @ R[j])
    # Gram-Schmidt adjoint
    g1, g2, g3 = gR[:, :, 0], gR[:, :, 1], gR[:, :, 2]
    g1 = g1 + np.cross(b2, g3)
    g2 = g2 + np.cross(g3, b1)
    gu = (g2 - np.sum(b2 * g2, -1, keepdims=True) * b2) / n2
    ga2 = gu - b1 * np.sum(b1 * gu, -1, keepdims=True)
    g1 = g1 - d12 * gu - a2 * np.sum(b1 * gu, -1, keepdims=True)
    ga1 = (g1 - np.sum(b1 * g1, -1, keepdims=True) * b1) / n1
    return L, np.concatenate([ga1, ga2, gt], axis=1)


# ------------------------------------------------------------------ residuals and IRLS

def residuals(theta: np.ndarray, pairs: np.ndarray, offsets: np.ndarray, uv: np.ndarray,
              block: int = 1 << 22) -> np.ndarray:
    """Algebraic epipolar residual r_nm = x2~^T E_n x1~ for every match [M].

    The matches are taken in runs of whole pairs of about `block` matches so
    that scenes of 10^8 matches fit in host memory; each residual is the same
    three-factor product either way."""
    E = essentials(theta, pairs)
    offsets = np.asarray(offsets, dtype=np.int64)
    counts = np.diff(offsets)
    P = counts.size
    out = np.zeros(int(offsets[-1]))
    n0 = 0
    while n0 < P:
        n1 = int(np.searchsorted(offsets, offsets[n0] + block, side="right")) - 1
        n1 = min(max(n1, n0 + 1), P)
        lo, hi = int(offsets[n0]), int(offsets[n1])
        En = np.repeat(E[n0:n1], counts[n0:n1], axis=0)
        x1, x2 = homogeneous(uv[lo:hi])
        out[lo:hi] = np.einsum("ma,mab,mb->m", x2, En, x1)
        n0 = n1
    return out


def irls_weights(r: np.ndarray, delta: float, tau: float) -> np.ndarray:
    """omega = 1/max(|r|, delta) where |r| <= tau, else 0 (reading R6)."""
    a = np.abs(r)
    return np.where(a <= tau, 1.0 / np.maximum(a, delta), 0.0)


# ------------------------------------------------------------------ Adam

def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-12):
    """One Adam update (Kingma & Ba, with bias correction); step counts from 1.
    lr may be a scalar or broadcastable to theta.  Returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


@dataclasses.dataclass
class Schedule:
    iters: int = 500            # total Adam steps
    round_len: int = 500        # steps per optimisation loop (reweight between loops)
    lr_rot: float = 3e-3        # initial lr on (a1, a2)
    lr_t: float = 1e-2          # initial lr on t
    lr_final_frac: float = 1e-3 # lr decays to lr0*frac over the solve
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-12
    irls: bool = False          # reweight between loops
    delta: float = 1e-4
    tau0: float = 0.1
    tau_min: float = 0.01
    first_round_unit_weights: bool = False
    reset_adam: bool = True     # restart Adam (m, v, step) at every loop


def lr_at(sched: Schedule, k: int) -> np.ndarray:
    """Per-parameter lr for global step k (0-based): exponential decay from lr0
    to lr0*frac over the whole solve (reading R5)."""
    f = sched.lr_final_frac ** (k / sched.iters)
    return np.array([sched.lr_rot] * 6 + [sched.lr_t] * 3) * f


def tau_at(sched: Schedule, k: int) -> float:
    """Filter threshold of the k-th reweighting (0-based): halves from tau0 to
    the floor tau_min (reading R6)."""
    return max(sched.tau0 * 0.5 ** k, sched.tau_min)


def solve(theta0: np.ndarray, pairs: np.ndarray, offsets: np.ndarray, uv: np.ndarray,
          sched: Schedule, weights0: np.ndarray | None = None, history: list | None = None,
          store=None):
    """Epipolar adjustment: loops of Adam steps on the weighted Gram form, with
    IRLS reweighting and outlier filtering between loops (Sec. 3.3).

    Returns (theta, loss trace, final weights).  If `history` is a list, one
    record per optimisation loop is appended to it: the loop index, the
    filter threshold its weights were computed with (None for unit or given
    weights), the poses they were computed at (None likewise), and Z.
    `store` (None: float64 throughout) is applied to theta after every Adam
    step: the precision the parameters are kept in between steps, all
    arithmetic staying float64 (e.g. rounding to float32 measures how far
    float32 parameter storage alone moves the solve).
    """
    theta = np.asarray(theta0, dtype=np.float64).copy()
    M = uv.shape[0]
    weights = weights0
    k_rw = 0
    rw_tau, rw_theta = None, None
    if weights is None and sched.irls and not sched.first_round_unit_weights:
        rw_tau, rw_theta = tau_at(sched, k_rw), theta.copy()
        weights = irls_weights(residuals(theta, pairs, offsets, uv), sched.delta, rw_tau)
        k_rw += 1
    trace = []
    done = 0
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    t_adam = 0
    loop = 0
    while done < sched.iters:
        W = pair_grams(uv, offsets, weights)
        Z = M if weights is None else int(np.count_nonzero(weights))
        if history is not None:
            history.append({"loop": loop, "tau": rw_tau, "theta": rw_theta, "Z": Z})
        loop += 1
        inv_Z = 1.0 / max(Z, 1)
        if sched.reset_adam:
            m = np.zeros_like(theta)
            v = np.zeros_like(theta)
            t_adam = 0
        K = min(sched.round_len, sched.iters - done)
        for s in range(K):
            L, g = loss_grad(theta, pairs, W, inv_Z)
            trace.append(L)
            t_adam += 1
            theta, m, v = adam_step(theta, g, m, v, t_adam, lr_at(sched, done + s),
                                    sched.beta1, sched.beta2, sched.eps)
            if store is not None:
                theta = store(theta)
        done += K
        if sched.irls and done < sched.iters:
            rw_tau, rw_theta = tau_at(sched, k_rw), theta.copy()
            weights = irls_weights(residuals(theta, pairs, offsets, uv), sched.delta, rw_tau)
            k_rw += 1
    return theta, np.array(trace), weights


# ------------------------------------------------------------------ pose comparison

def _angle_between_rotations(Ra, Rb):
    """Angle of Ra Rb^T in degrees: atan2(sin, cos) with sin from the
    skew part, accurate for small angles."""
    Q = Ra @ np.swapaxes(Rb, -1, -2)
    c = (np.trace(Q, axis1=-2, axis2=-1) - 1.0) / 2.0
    ax = np.stack([Q[:, 2, 1] - Q[:, 1, 2], Q[:, 0, 2] - Q[:, 2, 0], Q[:, 1, 0] - Q[:, 0, 1]], -1)
    return np.degrees(np.arctan2(0.5 * np.linalg.norm(ax, axis=-1), c))


def relative_pose_errors(theta_a: np.ndarray, theta_b: np.ndarray, pairs: np.ndarray):
    """Per-pair relative-rotation and relative-translation-direction errors in
    degrees between two solutions (RRA/RTA style, Sec. 4.1 metrics).  The
    epipolar objective cannot tell t from -t, so the translation error takes
    the better of the two global signs."""
    Ra, ta = poses_from_params(theta_a)
    Rb, tb = poses_from_params(theta_b)
    Rij_a, tij_a = relative(Ra, ta, pairs)
    Rij_b, tij_b = relative(Rb, tb, pairs)
    rot = _angle_between_rotations(Rij_a, Rij_b)
    ua = tij_a / np.linalg.norm(tij_a, axis=-1, keepdims=True)
    ub = tij_b / np.linalg.norm(tij_b, axis=-1, keepdims=True)
    c = np.sum(ua * ub, -1)
    sn = np.linalg.norm(np.cross(ua, ub), axis=-1)
    e_pos = np.degrees(np.arctan2(sn, c))
    e_neg = np.degrees(np.arctan2(sn, -c))
    trans = e_pos if e_pos.max() <= e_neg.max() else e_neg
    return rot, trans
