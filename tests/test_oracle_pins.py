"""Pins of the FP64 oracle against facts the paper and the mathematics fix.

None of these checks retypes an oracle formula: each compares the oracle with
an independent route (pure-Python brute force, the linear 8-point null vector,
the geometry that generated the data, invariances of the objective, central
finite differences, torch's own Adam) chosen so that a plausible slip in the
oracle (a dropped term, a transposed E, a wrong kron order, a sign) fails.
"""
import math

import numpy as np
import pytest
import torch

from oracle import ea
from paper_2505_04612_amd import synth


@pytest.fixture(scope="module")
def tiny():
    return synth.tiny()


@pytest.fixture(scope="module")
def tiny_clean():
    return synth.tiny(sigma=0.0, frac=0.0, init_trans="gt")


def _sub(scene, npairs=6, cap=120):
    """A few pairs of a scene, each cut to at most `cap` matches."""
    offs = [0]
    rows = []
    for n in range(npairs):
        lo, hi = scene.offsets[n], min(scene.offsets[n + 1], scene.offsets[n] + cap)
        rows.append(scene.uv[lo:hi])
        offs.append(offs[-1] + hi - lo)
    return np.concatenate(rows), np.array(offs, dtype=np.int64), scene.pairs[:npairs]


# ----------------------------------------------------------- Gram (App. B.6)

def test_gram_equals_bruteforce_epipolar_sum(tiny):
    """P1: sum_m omega (x2~^T E x1~)^2 (pure Python triple loop, no kron) equals
    e^T W e with the oracle's W, for random E and random weights."""
    uv, offs, _ = _sub(tiny)
    rng = np.random.default_rng(5)
    om = rng.uniform(0.1, 3.0, uv.shape[0])
    W = ea.pair_grams(uv, offs, om)
    for n in range(len(offs) - 1):
        E = rng.normal(size=(3, 3))
        brute = 0.0
        for m in range(offs[n], offs[n + 1]):
            x1 = (uv[m, 0], uv[m, 1], 1.0)
            x2 = (uv[m, 2], uv[m, 3], 1.0)
            r = 0.0
            for a in range(3):
                for b in range(3):
                    r += x2[a] * E[a][b] * x1[b]
            brute += om[m] * r * r
        e = E.reshape(9)
        q = float(e @ W[n] @ e)
        assert abs(q - brute) <= 1e-12 * abs(brute)


def test_gram_invariants(tiny):
    """P2: W symmetric PSD; W[8,8] = sum omega; tr W = sum omega |x2~|^2 |x1~|^2;
    entries depend only on the unordered index pairs {a,c}, {b,d} (36 distinct)."""
    uv, offs, _ = _sub(tiny, npairs=8, cap=400)
    rng = np.random.default_rng(6)
    om = rng.uniform(0.0, 2.0, uv.shape[0])
    W = ea.pair_grams(uv, offs, om)
    for n in range(len(offs) - 1):
        Wn = W[n]
        sl = slice(offs[n], offs[n + 1])
        assert np.array_equal(Wn, Wn.T) or np.allclose(Wn, Wn.T, rtol=0, atol=1e-12 * np.abs(Wn).max())
        ev = np.linalg.eigvalsh(Wn)
        assert ev.min() >= -1e-10 * ev.max()
        assert math.isclose(Wn[8, 8], om[sl].sum(), rel_tol=1e-13)
        n1 = uv[sl, 0] ** 2 + uv[sl, 1] ** 2 + 1.0
        n2 = uv[sl, 2] ** 2 + uv[sl, 3] ** 2 + 1.0
        assert math.isclose(np.trace(Wn), float(np.sum(om[sl] * n1 * n2)), rel_tol=1e-12)
        W4 = Wn.reshape(3, 3, 3, 3)           # [a, b, c, d]
        assert np.allclose(W4, W4.transpose(2, 1, 0, 3), rtol=1e-13, atol=0)
        assert np.allclose(W4, W4.transpose(0, 3, 2, 1), rtol=1e-13, atol=0)
        distinct = {tuple(sorted((a, c))) + tuple(sorted((b, d)))
                    for a in range(3) for b in range(3) for c in range(3) for d in range(3)}
        assert len(distinct) == 36


def test_gram_empty_pair_is_zero():
    uv = np.random.default_rng(0).normal(size=(10, 4))
    offs = np.array([0, 4, 4, 10], dtype=np.int64)
    W = ea.pair_grams(uv, offs)
    assert np.all(W[1] == 0.0)
    assert np.linalg.matrix_rank(W[0]) == 4


def test_null_vector_is_essential_matrix(tiny_clean):
    """P3: on noise-free data the smallest eigenvector of W_n (the linear
    8-point estimate) equals +-e_n computed by the oracle from the true poses.
    A transposed E, a swapped kron order or a wrong relative pose fails."""
    s = tiny_clean
    W = ea.pair_grams(s.uv, s.offsets)
    E = ea.essentials(ea.params_from_poses(s.R_gt, s.t_gt), s.pairs).reshape(-1, 9)
    for n in range(0, s.num_pairs, 7):
        ev, V = np.linalg.eigh(W[n])
        v = V[:, 0]
        e = E[n] / np.linalg.norm(E[n])
        assert min(np.linalg.norm(v - e), np.linalg.norm(v + e)) < 1e-6
        assert ev[0] <= 1e-12 * ev[-1]


def test_essential_singular_values(tiny):
    """E = [t_hat]_x R has singular values (1, 1, 0) for unit t_hat."""
    th = ea.params_from_poses(tiny.R_init, tiny.t_init)
    E = ea.essentials(th, tiny.pairs)
    sv = np.linalg.svd(E, compute_uv=False)
    assert np.allclose(sv[:, 0], 1.0, atol=1e-12)
    assert np.allclose(sv[:, 1], 1.0, atol=1e-12)
    assert np.allclose(sv[:, 2], 0.0, atol=1e-12)


# ----------------------------------------------------------- loss (eq. epipolar-objective-l2)

def test_zero_residual_and_loss_at_ground_truth(tiny_clean):
    """P4: every match satisfies the epipolar constraint at the true poses on
    noise-free data (the geometry the generator projected), so the loss is at
    the float64 cancellation floor."""
    s = tiny_clean
    th = ea.params_from_poses(s.R_gt, s.t_gt)
    r = ea.residuals(th, s.pairs, s.offsets, s.uv)
    assert np.abs(r).max() <= 1e-12
    W = ea.pair_grams(s.uv, s.offsets)
    e = ea.essentials(th, s.pairs).reshape(-1, 9)
    per_pair = ea.pair_losses(th, s.pairs, W)
    floor = 1e-12 * np.linalg.norm(W.reshape(len(W), -1), axis=1) * np.sum(e * e, axis=1)
    assert np.all(np.abs(per_pair) <= floor)


def test_l2_form_equals_mean_square_residual(tiny):
    """The quadratic form is the per-match mean of squared epipolar errors
    (reading: no factor 2), computed here from the per-match residuals."""
    th = ea.params_from_poses(tiny.R_init, tiny.t_init)
    W = ea.pair_grams(tiny.uv, tiny.offsets)
    r = ea.residuals(th, tiny.pairs, tiny.offsets, tiny.uv)
    L = ea.loss_from_grams(th, tiny.pairs, W, 1.0 / tiny.num_matches)
    assert math.isclose(L, float(np.mean(r * r)), rel_tol=1e-11)


def _similarity(theta, seed):
    """Apply a world similarity X' = s G X + c to the poses."""
    rng = np.random.default_rng(seed)
    A = rng.normal(size=(3, 3))
    G, _ = np.linalg.qr(A)
    if np.linalg.det(G) < 0:
        G[:, 0] = -G[:, 0]
    c = rng.normal(size=3) * 3.0
    s = float(rng.uniform(0.2, 5.0))
    R, t = ea.poses_from_params(theta)
    R2 = R @ G.T
    t2 = s * t - np.einsum("nab,b->na", R2, c)
    return ea.params_from_poses(R2, t2)


def test_loss_invariant_under_similarity(tiny):
    """P6: a global rotation, offset and scale of the world leaves L unchanged."""
    th = ea.params_from_poses(tiny.R_init, tiny.t_init)
    rng = np.random.default_rng(1)
    om = rng.uniform(0.5, 2.0, tiny.num_matches)
    W = ea.pair_grams(tiny.uv, tiny.offsets, om)
    L0 = ea.loss_from_grams(th, tiny.pairs, W, 1e-3)
    for seed in range(3):
        L1 = ea.loss_from_grams(_similarity(th, seed), tiny.pairs, W, 1e-3)
        assert math.isclose(L0, L1, rel_tol=1e-12)


def test_gram_schmidt_roundtrip_and_orthonormality():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(50, 3, 3))
    Q, _ = np.linalg.qr(A)
    Q[np.linalg.det(Q) < 0, :, 0] *= -1
    R = ea.rot_from_6d(Q[:, :, 0], Q[:, :, 1])
    assert np.allclose(R, Q, atol=1e-14)
    a1 = rng.normal(size=(50, 3)) * 3
    a2 = rng.normal(size=(50, 3)) * 0.3
    R = ea.rot_from_6d(a1, a2)
    assert np.allclose(np.swapaxes(R, 1, 2) @ R, np.eye(3), atol=1e-14)
    assert np.allclose(np.linalg.det(R), 1.0, atol=1e-14)


# ----------------------------------------------------------- gradient

def _fd_check(th, pairs, W, inv_Z, seed, ndir=8):
    L, g = ea.loss_grad(th, pairs, W, inv_Z)
    assert math.isclose(L, ea.loss_from_grams(th, pairs, W, inv_Z), rel_tol=1e-13)
    rng = np.random.default_rng(seed)
    for _ in range(ndir):
        d = rng.normal(size=th.shape)
        h = 1e-6 * max(1.0, float(np.abs(th).max()))
        fd = (ea.loss_from_grams(th + h * d, pairs, W, inv_Z)
              - ea.loss_from_grams(th - h * d, pairs, W, inv_Z)) / (2 * h)
        an = float(np.sum(g * d))
        assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-300) + 1e-7 * float(np.linalg.norm(g) * np.linalg.norm(d))


def test_gradient_matches_central_differences(tiny):
    """P7: analytic chain rule vs central differences in float64."""
    th = ea.params_from_poses(tiny.R_init, tiny.t_init)
    # perturb the 6D parameters off the orthonormal manifold so the
    # Gram-Schmidt adjoint is exercised in full
    rng = np.random.default_rng(2)
    th = th + rng.normal(0, 0.05, th.shape)
    om = rng.uniform(0.2, 2.0, tiny.num_matches)
    W = ea.pair_grams(tiny.uv, tiny.offsets, om)
    _fd_check(th, tiny.pairs, W, 1.0 / tiny.num_matches, seed=4)


def test_gradient_per_coordinate(tiny):
    th = ea.params_from_poses(tiny.R_init, tiny.t_init)
    W = ea.pair_grams(tiny.uv, tiny.offsets)
    L, g = ea.loss_grad(th, tiny.pairs, W, 1e-4)
    h = 1e-6
    for (c, k) in [(0, 0), (3, 4), (7, 8), (19, 2), (11, 6)]:
        tp = th.copy(); tp[c, k] += h
        tm = th.copy(); tm[c, k] -= h
        fd = (ea.loss_from_grams(tp, tiny.pairs, W, 1e-4) - ea.loss_from_grams(tm, tiny.pairs, W, 1e-4)) / (2 * h)
        assert abs(fd - g[c, k]) <= 1e-7 * np.abs(g).max()


def test_gradient_zero_along_gauge(tiny):
    """The loss is invariant under a global similarity, so the gradient has no
    component along an infinitesimal global translation or scale."""
    th = ea.params_from_poses(tiny.R_init, tiny.t_init)
    W = ea.pair_grams(tiny.uv, tiny.offsets)
    L, g = ea.loss_grad(th, tiny.pairs, W, 1e-4)
    R, t = ea.poses_from_params(th)
    d_scale = np.zeros_like(th); d_scale[:, 6:9] = t
    c = np.array([0.3, -1.0, 0.7])
    d_shift = np.zeros_like(th); d_shift[:, 6:9] = -np.einsum("nab,b->na", R, c)
    scale = np.linalg.norm(g) * np.linalg.norm(t)
    assert abs(np.sum(g * d_scale)) <= 1e-10 * scale
    assert abs(np.sum(g * d_shift)) <= 1e-10 * scale


def test_pair_rotation_gradients_are_opposite_in_body_frames(tiny):
    """A pair's loss depends on R_i, R_j only through R_ij = R_j R_i^T, so a
    common body-frame turn R -> R exp([d]_x) of both cameras leaves it
    unchanged: the rate along d of camera i's parameters is minus that of
    camera j's, pair by pair (what lets the fused loops exchange one
    rotation term per pair).  Rates from the oracle's analytic gradient."""
    th = ea.params_from_poses(tiny.R_init, tiny.t_init)
    W = ea.pair_grams(tiny.uv, tiny.offsets)
    R, _ = ea.poses_from_params(th)
    rng = np.random.default_rng(5)
    for n in range(0, tiny.num_pairs, 17):
        pair = tiny.pairs[n:n + 1]
        _, g = ea.loss_grad(th, pair, W[n:n + 1], 1e-3)
        for _ in range(3):
            d = ea.skew(rng.normal(size=3))
            rate = []
            for c in pair[0]:
                dR = R[c] @ d           # d/d(eps) of R exp(eps [d]_x); a1, a2 are R's first two columns
                rate.append(np.dot(g[c, 0:3], dR[:, 0]) + np.dot(g[c, 3:6], dR[:, 1]))
            scale = np.linalg.norm(g[pair[0], 0:6]) * np.linalg.norm(d)
            assert abs(rate[0] + rate[1]) <= 1e-10 * scale, (n, rate)
            assert abs(rate[0]) > 1e-6 * scale or scale == 0.0


def test_gradient_zero_where_rotation_does_not_move(tiny):
    """Scaling a1 or a2 and adding a multiple of a1 to a2 leave R = GS(a1, a2)
    unchanged, so the gradient has no component along them: only the tangent
    part of dL/dR reaches the 6D parameters."""
    rng = np.random.default_rng(6)
    th = ea.params_from_poses(tiny.R_init, tiny.t_init)
    th[:, 0:3] *= rng.uniform(0.5, 2.0, (tiny.num_cams, 1))
    th[:, 3:6] = th[:, 3:6] * rng.uniform(0.5, 2.0, (tiny.num_cams, 1)) + 0.3 * th[:, 0:3]
    W = ea.pair_grams(tiny.uv, tiny.offsets)
    _, g = ea.loss_grad(th, tiny.pairs, W, 1e-3)
    a1, a2 = th[:, 0:3], th[:, 3:6]
    scale = np.linalg.norm(g[:, 0:6], axis=1) * np.maximum(np.linalg.norm(a1, axis=1), np.linalg.norm(a2, axis=1))
    for d1, d2 in ((a1, 0 * a2), (0 * a1, a1), (0 * a1, a2)):
        rate = np.sum(g[:, 0:3] * d1, axis=1) + np.sum(g[:, 3:6] * d2, axis=1)
        assert np.all(np.abs(rate) <= 1e-10 * scale + 1e-300)


# ----------------------------------------------------------- IRLS

def test_irls_weighted_l2_equals_l1_at_reweight_point(tiny):
    """P5: at the poses where the weights were computed, the weighted L2 loss
    equals the L1 loss over kept matches with |r| >= delta, and its gradient
    equals twice the L1 subgradient."""
    th = ea.params_from_poses(tiny.R_init, tiny.t_init)
    r = ea.residuals(th, tiny.pairs, tiny.offsets, tiny.uv)
    delta, tau = 1e-4, 0.05
    w = ea.irls_weights(r, delta, tau)
    kept = w > 0
    assert np.all(np.abs(r[kept]) <= tau) and np.all(np.abs(r[~kept]) > tau)
    Z = int(kept.sum())
    W = ea.pair_grams(tiny.uv, tiny.offsets, w)
    L2w = ea.loss_from_grams(th, tiny.pairs, W, 1.0 / Z)
    big = kept & (np.abs(r) >= delta)
    small = kept & (np.abs(r) < delta)
    L1 = (np.abs(r[big]).sum() + (r[small] ** 2).sum() / delta) / Z
    assert math.isclose(L2w, L1, rel_tol=1e-10)
    # gradient: d(omega r^2) = 2 sign(r) dr = 2 d|r| where |r| >= delta, and
    # d(r^2/delta) below the floor
    _, g = ea.loss_grad(th, tiny.pairs, W, 1.0 / Z)
    rng = np.random.default_rng(9)
    d = rng.normal(size=th.shape)
    h = 1e-7
    rp = ea.residuals(th + h * d, tiny.pairs, tiny.offsets, tiny.uv)
    rm = ea.residuals(th - h * d, tiny.pairs, tiny.offsets, tiny.uv)
    fd_big = (np.abs(rp[big]).sum() - np.abs(rm[big]).sum()) / (2 * h) / Z
    fd_small = ((rp[small] ** 2).sum() - (rm[small] ** 2).sum()) / delta / (2 * h) / Z
    an = float(np.sum(g * d))
    assert abs(an - (2 * fd_big + fd_small)) <= 1e-6 * abs(an)


def test_irls_weight_rule():
    r = np.array([0.0, 5e-5, -1e-4, 2e-3, -0.05, 0.0500001, -1.0])
    w = ea.irls_weights(r, 1e-4, 0.05)
    assert np.array_equal(w, np.array([1e4, 1e4, 1e4, 500.0, 20.0, 0.0, 0.0]))


# ----------------------------------------------------------- Adam

def test_adam_matches_torch_adam():
    """P8: the oracle's Adam equals torch.optim.Adam (float64, CPU) on the same
    gradient sequence with a changing learning rate."""
    rng = np.random.default_rng(11)
    p0 = rng.normal(size=(7, 9))
    grads = [rng.normal(size=(7, 9)) * 10.0 ** rng.uniform(-6, 1) for _ in range(25)]
    lrs = [1e-2 * 0.9 ** k for k in range(25)]
    p = torch.tensor(p0.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=lrs[0], betas=(0.9, 0.999), eps=1e-12)
    th, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for k, g in enumerate(grads):
        for grp in opt.param_groups:
            grp["lr"] = lrs[k]
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        th, m, v = ea.adam_step(th, g, m, v, k + 1, lrs[k], 0.9, 0.999, 1e-12)
    assert np.allclose(th, p.detach().numpy(), rtol=0, atol=1e-14)


def test_lr_schedule_endpoints():
    s = ea.Schedule(iters=200, lr_rot=2e-3, lr_t=1e-2, lr_final_frac=1e-3)
    assert np.allclose(ea.lr_at(s, 0), [2e-3] * 6 + [1e-2] * 3)
    assert np.allclose(ea.lr_at(s, 200), [2e-6] * 6 + [1e-5] * 3)
    assert np.allclose(ea.lr_at(s, 100), np.sqrt(ea.lr_at(s, 0) * ea.lr_at(s, 200)))


def test_tau_schedule():
    s = ea.Schedule(tau0=0.1, tau_min=0.01)
    assert [ea.tau_at(s, k) for k in range(6)] == [0.1, 0.05, 0.025, 0.0125, 0.01, 0.01]


# ----------------------------------------------------------- whole solve

def test_solve_converges_to_ground_truth_noise_free(tiny_clean):
    """P9: from the true poses with 1 deg rotation noise on noise-free data the
    solve returns to the truth up to gauge."""
    s = tiny_clean
    R1, t1 = synth._init_poses(s.R_gt, s.t_gt, 0, rot_deg=1.0, trans="gt")
    th0 = ea.params_from_poses(R1, t1)
    th_gt = ea.params_from_poses(s.R_gt, s.t_gt)
    sched = ea.Schedule(iters=1000, round_len=1000, lr_rot=3e-3, lr_t=9e-3, lr_final_frac=1e-3)
    th, trace, _ = ea.solve(th0, s.pairs, s.offsets, s.uv, sched)
    rot, tra = ea.relative_pose_errors(th, th_gt, s.pairs)
    assert rot.max() < 0.01
    assert tra.max() < 0.2
    assert trace[-1] < 1e-5 * trace[0]


@pytest.fixture(scope="module")
def tiny_outliers():
    return synth.tiny(sigma=0.0, frac=0.2, init_trans="gt")


def test_irls_solve_rejects_outliers(tiny_outliers):
    """The IRLS branch of the solve (Sec. 3.3, the IRLS and filtering
    paragraph): on noise-free matches with 20 % outliers, from the true poses
    with 1 deg rotation noise, reweighting and filtering between loops return
    the solve to the truth, while the same schedule without reweighting (plain
    L2 over every match) is pulled far away by the outliers."""
    s = tiny_outliers
    assert 0.15 < s.outlier.mean() < 0.25
    R1, t1 = synth._init_poses(s.R_gt, s.t_gt, 0, rot_deg=1.0, trans="gt")
    th0 = ea.params_from_poses(R1, t1)
    th_gt = ea.params_from_poses(s.R_gt, s.t_gt)
    errs = {}
    for irls in (True, False):
        sched = ea.Schedule(iters=1000, round_len=100, lr_rot=3e-3, lr_t=9e-3, lr_final_frac=1e-3, irls=irls)
        th, _, w = ea.solve(th0, s.pairs, s.offsets, s.uv, sched)
        errs[irls] = ea.relative_pose_errors(th, th_gt, s.pairs)
        if irls:
            # the final filter (tau_min = 0.01) drops most outliers and no inlier
            assert np.all(w[~s.outlier] > 0)
            assert np.count_nonzero(w[s.outlier]) < 0.2 * s.outlier.sum()
    assert errs[True][0].max() < 0.01 and errs[True][1].max() < 0.1
    assert errs[False][0].max() > 1.0


def test_irls_loop_records_against_hand_count(tiny_outliers):
    """Loop by loop: the first loop's weights come from the initial poses
    (reading R8), each later loop's from the poses the previous loop ended at;
    the filter threshold is tau0 halved per reweighting down to tau_min
    (0.1, 0.05, 0.025, 0.0125, 0.01, 0.01); Z equals a hand count of the
    matches with |r| <= tau at those poses.  One loop is replayed by hand from
    the oracle's pinned pieces (Gram, loss gradient, Adam)."""
    s = tiny_outliers
    R1, t1 = synth._init_poses(s.R_gt, s.t_gt, 0, rot_deg=2.0, trans="gt")
    th0 = ea.params_from_poses(R1, t1)
    sched = ea.Schedule(iters=600, round_len=100, lr_rot=3e-3, lr_t=9e-3, lr_final_frac=1e-3, irls=True)
    hist = []
    th, trace, w = ea.solve(th0, s.pairs, s.offsets, s.uv, sched, history=hist)
    assert [h["loop"] for h in hist] == list(range(6))
    assert [h["tau"] for h in hist] == [0.1, 0.05, 0.025, 0.0125, 0.01, 0.01]
    assert np.array_equal(hist[0]["theta"], th0)
    for h in hist:
        r = ea.residuals(h["theta"], s.pairs, s.offsets, s.uv)
        count = 0
        for x in r.tolist():
            if abs(x) <= h["tau"]:
                count += 1
        assert h["Z"] == count
    assert np.count_nonzero(w) == hist[-1]["Z"]
    assert len(trace) == 600
    # loop 0 by hand: weights at th0, Gram, 100 Adam steps from zero moments
    w0 = np.where(np.abs(ea.residuals(th0, s.pairs, s.offsets, s.uv)) <= 0.1,
                  1.0 / np.maximum(np.abs(ea.residuals(th0, s.pairs, s.offsets, s.uv)), 1e-4), 0.0)
    W = ea.pair_grams(s.uv, s.offsets, w0)
    x, m, v = th0.copy(), np.zeros_like(th0), np.zeros_like(th0)
    for k in range(100):
        L, g = ea.loss_grad(x, s.pairs, W, 1.0 / np.count_nonzero(w0))
        assert L == trace[k]
        x, m, v = ea.adam_step(x, g, m, v, k + 1, ea.lr_at(sched, k))
    assert np.array_equal(x, hist[1]["theta"])
    # unit weights in the first loop: Z = M there, thresholds start one loop later
    hist_u = []
    sched_u = ea.Schedule(iters=300, round_len=100, irls=True, first_round_unit_weights=True)
    ea.solve(th0, s.pairs, s.offsets, s.uv, sched_u, history=hist_u)
    assert [h["tau"] for h in hist_u] == [None, 0.1, 0.05]
    assert hist_u[0]["Z"] == s.num_matches and hist_u[0]["theta"] is None


def test_relative_pose_errors_pin():
    """The pose metric sees a known rotation of one camera and ignores a global
    similarity and the global sign of t."""
    s = synth.tiny(sigma=0.0, frac=0.0)
    th = ea.params_from_poses(s.R_gt, s.t_gt)
    rot, tra = ea.relative_pose_errors(th, _similarity(th, 4), s.pairs)
    assert rot.max() < 1e-9 and tra.max() < 1e-9
    flipped = th.copy(); flipped[:, 6:9] *= -1.0
    rot, tra = ea.relative_pose_errors(th, flipped, s.pairs)
    assert rot.max() < 1e-9 and tra.max() < 1e-9
    R, t = ea.poses_from_params(th)
    G = synth._axis_angle(np.array([[0.0, 0.0, 1.0]]), np.array([np.deg2rad(2.0)]))[0]
    R2 = R.copy(); R2[5] = G @ R[5]
    t2 = t.copy(); t2[5] = G @ t[5]       # same centre, rotated camera
    rot, tra = ea.relative_pose_errors(th, ea.params_from_poses(R2, t2), s.pairs)
    touching = (s.pairs[:, 0] == 5) | (s.pairs[:, 1] == 5)
    assert np.allclose(rot[touching], 2.0, atol=1e-9)
    assert rot[~touching].max() < 1e-9


# ----------------------------------------------------------- planted mistakes

def test_pins_catch_planted_mistakes(tiny_clean, monkeypatch):
    """Plant plausible slips in the oracle (on the CPU) and check that the
    pins above would fail for each."""
    s = tiny_clean
    th = ea.params_from_poses(s.R_gt, s.t_gt)
    W = ea.pair_grams(s.uv, s.offsets)
    good = ea.essentials(th, s.pairs).reshape(-1, 9)[0]

    def null_vec_ok():
        v = np.linalg.eigh(W[0])[1][:, 0]
        e = ea.essentials(th, s.pairs).reshape(-1, 9)[0]
        e = e / np.linalg.norm(e)
        return min(np.linalg.norm(v - e), np.linalg.norm(v + e)) < 1e-6

    assert null_vec_ok()
    orig = ea.essentials
    monkeypatch.setattr(ea, "essentials", lambda t, p: np.swapaxes(orig(t, p), -1, -2))
    assert not null_vec_ok()                         # transposed E
    monkeypatch.setattr(ea, "essentials", orig)
    orig_rel = ea.relative
    monkeypatch.setattr(ea, "relative", lambda R, t, p: (R[p[:, 1]] @ np.swapaxes(R[p[:, 0]], -1, -2),
                                                         t[p[:, 1]] - t[p[:, 0]]))
    assert not null_vec_ok()                         # dropped R_ij t_i term
    monkeypatch.setattr(ea, "relative", orig_rel)
    # kron order swapped in the Gram: the brute-force identity breaks
    orig_mv = ea.match_vectors
    monkeypatch.setattr(ea, "match_vectors",
                        lambda uv: orig_mv(np.ascontiguousarray(uv[:, [2, 3, 0, 1]])))
    W_bad = ea.pair_grams(s.uv[:50], np.array([0, 50]))
    monkeypatch.setattr(ea, "match_vectors", orig_mv)
    E = np.random.default_rng(0).normal(size=(3, 3))
    x1, x2 = ea.homogeneous(s.uv[:50])
    brute = float(np.sum(np.einsum("ma,ab,mb->m", x2, E, x1) ** 2))
    assert not math.isclose(float(E.reshape(9) @ W_bad[0] @ E.reshape(9)), brute, rel_tol=1e-6)
    assert np.linalg.norm(good) > 0


def test_irls_pins_catch_planted_mistakes(tiny_outliers, monkeypatch):
    """Plant slips in the IRLS branch (on the CPU): a threshold that never
    decays and a filter that keeps every match; the loop records then
    disagree with the hand count / the printed threshold sequence."""
    s = tiny_outliers
    th0 = ea.params_from_poses(s.R_gt, s.t_gt)
    sched = ea.Schedule(iters=300, round_len=100, irls=True)

    def records():
        hist = []
        ea.solve(th0, s.pairs, s.offsets, s.uv, sched, history=hist)
        return hist

    def hand_ok(hist):
        taus_ok = [h["tau"] for h in hist] == [0.1, 0.05, 0.025]
        z_ok = all(h["Z"] == int(np.sum(np.abs(ea.residuals(h["theta"], s.pairs, s.offsets, s.uv)) <= tau))
                   for h, tau in zip(hist, [0.1, 0.05, 0.025]))
        return taus_ok and z_ok

    assert hand_ok(records())
    orig_tau = ea.tau_at
    monkeypatch.setattr(ea, "tau_at", lambda sc, k: sc.tau0)
    assert not hand_ok(records())                    # threshold never decays
    monkeypatch.setattr(ea, "tau_at", orig_tau)
    orig_w = ea.irls_weights
    monkeypatch.setattr(ea, "irls_weights", lambda r, d, t: 1.0 / np.maximum(np.abs(r), d))
    assert not hand_ok(records())                    # no outlier filter
    monkeypatch.setattr(ea, "irls_weights", orig_w)


# ----------------------------------------------------------- learned-weight MLP

def test_mlp_backward_matches_central_differences():
    from oracle import mlp
    rng = np.random.default_rng(21)
    p = mlp.init_params(3)
    for k in p:
        p[k] = p[k] + rng.normal(0, 0.05, p[k].shape)
    feats = rng.normal(size=(40, 3)) * [2.0, 1.0, 0.1] + [-6.0, 5.0, 0.2]
    mean, std = np.array([-6.0, 5.0, 0.2]), np.array([2.0, 1.0, 0.1])
    dout = rng.normal(size=40)
    g = mlp.backward(p, feats, mean, std, dout)
    h = 1e-6
    for k, shape in mlp.SHAPES.items():
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in shape)
            pp = {q: v.copy() for q, v in p.items()}
            pm = {q: v.copy() for q, v in p.items()}
            pp[k][idx] += h
            pm[k][idx] -= h
            fd = (np.sum(dout * mlp.forward(pp, feats, mean, std)[0])
                  - np.sum(dout * mlp.forward(pm, feats, mean, std)[0])) / (2 * h)
            assert abs(fd - g[k][idx]) <= 1e-6 * max(1.0, abs(fd)), (k, idx, fd, g[k][idx])


def test_mlp_closed_forms():
    """Zero weights give sigmoid(b3); a single active path gives the product
    of its weights."""
    from oracle import mlp
    p = {k: np.zeros(s) for k, s in mlp.SHAPES.items()}
    p["b3"][0] = 0.3
    f = np.random.default_rng(0).normal(size=(5, 3))
    out, _ = mlp.forward(p, f, np.zeros(3), np.ones(3))
    assert np.allclose(out, 1.0 / (1.0 + np.exp(-0.3)))
    p["W1"][7, 2] = 2.0
    p["W2"][11, 7] = 0.5
    p["W3"][0, 11] = 3.0
    f = np.array([[0.0, 0.0, 1.5], [0.0, 0.0, -1.0]])
    out, _ = mlp.forward(p, f, np.zeros(3), np.ones(3))
    z = np.array([0.3 + 3.0 * 0.5 * 2.0 * 1.5, 0.3])
    assert np.allclose(out, 1.0 / (1.0 + np.exp(-z)))


def test_match_features_closed_form():
    """Two cameras looking down +z, the second shifted by b along x: a point
    at depth D straight ahead of camera 1 has parallax atan(b/D), zero
    residual at the true poses, and f1 = log(#matches)."""
    from oracle import mlp
    b, D = 0.5, 4.0
    R = np.stack([np.eye(3), np.eye(3)])
    t = np.array([[0.0, 0.0, 0.0], [-b, 0.0, 0.0]])
    th = ea.params_from_poses(R, t)
    X = np.array([[0.0, 0.0, D], [0.3, -0.2, 2.0 * D]])
    uv = np.stack([X[:, 0] / X[:, 2], X[:, 1] / X[:, 2], (X[:, 0] - b) / X[:, 2], X[:, 1] / X[:, 2]], axis=1)
    f = mlp.features(th, np.array([[0, 1]]), np.array([0, 2]), uv, 1e-4)
    assert np.allclose(f[:, 0], np.log(1e-4))
    assert np.allclose(f[:, 1], np.log(2.0))
    assert np.isclose(f[0, 2], np.arctan2(b, D), atol=1e-12)
    c2 = np.array([b, 0.0, 0.0])
    a1, a2 = X[1], X[1] - c2
    ang = np.arccos(a1 @ a2 / np.linalg.norm(a1) / np.linalg.norm(a2))
    assert np.isclose(f[1, 2], ang, atol=1e-9)
