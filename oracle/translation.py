"""FP64 CPU oracle for FastMap's global translation averaging (arXiv 2505.04612).

TEST INFRASTRUCTURE ONLY.  The plain, slow, obviously correct reference the
HIP translation-averaging calls are checked against.  Only the tests, the
package's smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does.  It imports nothing from the package (only the Adam
step of the epipolar oracle) and computes in float64 with NumPy.

What it follows:
  * Sec. 3.3 "Global Translation": the target direction of pair (i, j) is
    o^{i->j} = -R_j^T t^{i->j} for world-to-camera R_j and the unit relative
    translation t^{i->j}; the camera centres o minimise
        L_t = (1/|P|) sum_(i,j) || (o_j - o_i)/|o_j - o_i| - o^{i->j} ||_1
    (eq. global-translation-objective) by first-order descent from a random
    initialisation;
  * App. "Multiple Initializations": several independent runs; each run is
    aligned by moving its centroid to the origin and scaling it to unit
    average norm; every camera takes its position from the run whose average
    loss for that camera is lowest; the merged centres initialise a final
    optimisation loop.

Readings where the paper is silent (each also listed in the design notes):
  T1  the subgradient of |x| at x = 0 is taken as 0 (sign(0) = 0);
  T2  a pair whose two centres coincide has no direction: it adds nothing to
      the loss or the gradient (the mean still divides by |P|);
  T3  the optimiser is Adam (the paper's first-order method, Sec. 3.2), with
      the learning rate decaying exponentially from lr0 to lr0*frac over the
      K steps of a loop, and fresh moments at the start of every loop;
  T4  a camera's average loss is the mean, over the pairs that contain it, of
      that pair's L1 term, on the run's own (unaligned) solution - the term is
      invariant to the alignment; a camera in no pair scores 0 in every run;
      among equal scores the lowest run index wins;
  T5  "unit average norm" is the mean of |o_i - centroid| over all cameras; a
      run whose centres all coincide (mean norm 0) is only centred.
"""
from __future__ import annotations

import numpy as np

from .ea import adam_step


# ------------------------------------------------------------------ target directions

def target_directions(R: np.ndarray, t_rel: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """o^{i->j} = -R_j^T t^{i->j} per pair (Sec. 3.3, Global Translation).
    R [N,3,3] world-to-camera rotations, t_rel [P,3], pairs [P,2] -> [P,3]."""
    R = np.asarray(R, dtype=np.float64)
    t_rel = np.asarray(t_rel, dtype=np.float64)
    Rj = R[np.asarray(pairs)[:, 1]]
    return -np.einsum("pba,pb->pa", Rj, t_rel)


# ------------------------------------------------------------------ objective

def pair_terms(o: np.ndarray, pairs: np.ndarray, d: np.ndarray):
    """Per pair: s = o_j - o_i, |s|, the unit direction u (0 where |s| = 0) and
    the L1 term |u - d|_1 (0 where |s| = 0, reading T2)."""
    o = np.asarray(o, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    pairs = np.asarray(pairs)
    s = o[pairs[:, 1]] - o[pairs[:, 0]]
    ns = np.linalg.norm(s, axis=1)
    live = ns > 0.0
    u = np.zeros_like(s)
    u[live] = s[live] / ns[live, None]
    term = np.where(live, np.abs(u - d).sum(axis=1), 0.0)
    return s, ns, u, term, live


def loss(o: np.ndarray, pairs: np.ndarray, d: np.ndarray) -> float:
    """L_t (eq. global-translation-objective)."""
    P = len(pairs)
    if P == 0:
        return 0.0
    return float(pair_terms(o, pairs, d)[3].sum() / P)


def loss_grad(o: np.ndarray, pairs: np.ndarray, d: np.ndarray):
    """(L_t, dL_t/do [N,3]).  Chain rule through the normalisation:
    dL/du = sign(u - d)/|P|, dL/ds = (I - u u^T) dL/du / |s|, and s = o_j - o_i
    gives +dL/ds to camera j and -dL/ds to camera i."""
    o = np.asarray(o, dtype=np.float64)
    P = len(pairs)
    g = np.zeros_like(o)
    if P == 0:
        return 0.0, g
    s, ns, u, term, live = pair_terms(o, pairs, d)
    gu = np.sign(u - d) / P
    gs = np.zeros_like(s)
    gs[live] = (gu[live] - u[live] * (u[live] * gu[live]).sum(axis=1, keepdims=True)) / ns[live, None]
    pairs = np.asarray(pairs)
    np.add.at(g, pairs[:, 1], gs)
    np.add.at(g, pairs[:, 0], -gs)
    return float(term.sum() / P), g


# ------------------------------------------------------------------ optimisation loop

def lr_at(lr0: float, frac: float, K: int, k: int) -> float:
    """Learning rate of step k (0-based) of a K-step loop (reading T3)."""
    return lr0 * frac ** (k / K)


def solve(o0: np.ndarray, pairs: np.ndarray, d: np.ndarray, K: int, lr0: float = 1e-2,
          frac: float = 1e-2, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-12):
    """K Adam steps on L_t from centres o0 [N,3]; returns (o, loss trace [K])
    where the trace holds L_t before each update."""
    o = np.array(o0, dtype=np.float64)
    m = np.zeros_like(o)
    v = np.zeros_like(o)
    trace = np.zeros(K)
    for k in range(K):
        trace[k], g = loss_grad(o, pairs, d)
        o, m, v = adam_step(o, g, m, v, k + 1, lr_at(lr0, frac, K, k), beta1, beta2, eps)
    return o, trace


# ------------------------------------------------------------------ multiple initialisations

def normalize(o: np.ndarray) -> np.ndarray:
    """Centroid to the origin, then unit average norm (reading T5)."""
    o = np.asarray(o, dtype=np.float64)
    c = o - o.mean(axis=0)
    scale = np.linalg.norm(c, axis=1).mean() if len(o) else 0.0
    return c / scale if scale > 0.0 else c


def camera_losses(o: np.ndarray, pairs: np.ndarray, d: np.ndarray, N: int) -> np.ndarray:
    """Average L1 term of the pairs containing each camera [N] (reading T4)."""
    term = pair_terms(o, pairs, d)[3]
    pairs = np.asarray(pairs)
    tot = np.zeros(N)
    cnt = np.zeros(N)
    for side in (0, 1):
        np.add.at(tot, pairs[:, side], term)
        np.add.at(cnt, pairs[:, side], 1.0)
    return np.where(cnt > 0, tot / np.maximum(cnt, 1.0), 0.0)


def merge(runs: np.ndarray, pairs: np.ndarray, d: np.ndarray):
    """Merge R runs [R,N,3] (App. Multiple Initializations).  Returns
    (merged centres [N,3], chosen run per camera [N], camera losses [R,N])."""
    runs = np.asarray(runs, dtype=np.float64)
    R, N = runs.shape[0], runs.shape[1]
    cam = np.stack([camera_losses(runs[r], pairs, d, N) for r in range(R)])
    choice = np.argmin(cam, axis=0)              # first minimum: lowest run index
    aligned = np.stack([normalize(runs[r]) for r in range(R)])
    merged = aligned[choice, np.arange(N)]
    return merged, choice, cam


def averaging(o_init: np.ndarray, pairs: np.ndarray, d: np.ndarray, K: int, K_final: int,
              lr0: float = 1e-2, frac: float = 1e-2):
    """The whole stage: R independent runs from o_init [R,N,3], the merge, and a
    final loop from the merged centres.  Returns (centres [N,3], info)."""
    runs = np.stack([solve(o_init[r], pairs, d, K, lr0, frac)[0] for r in range(len(o_init))])
    merged, choice, cam = merge(runs, pairs, d)
    o, trace = solve(merged, pairs, d, K_final, lr0, frac)
    return o, {"runs": runs, "merged": merged, "choice": choice, "cam_loss": cam, "trace": trace}
