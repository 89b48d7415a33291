"""Rotation averaging on the GPU (Sec. 3.3 "Global Rotation"; appendix on
rotation initialisation) against the FP64 oracle on the same stored inputs:
loss and gradient, the fused persistent loop, and its endpoint."""
import numpy as np
import pytest
import torch

from oracle import rotation as ra
from paper_2505_04612_amd import synth
from tests import helpers

pytestmark = pytest.mark.gpu


def _ctx():
    from paper_2505_04612_amd import api
    return api.default_context()


def _f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def _graph_scene(ctx, N, pairs):
    from paper_2505_04612_amd import api
    P = len(pairs)
    return api.Scene.from_numpy(ctx, N, pairs, np.zeros(P + 1, np.int64), np.zeros((0, 4)), torch.float32)


def _params(R):
    return np.concatenate([R[:, :, 0], R[:, :, 1]], axis=1)


def _perturbed(sc, seed, scale=0.05):
    rng = np.random.default_rng(seed)
    return (_params(sc.R_gt) + scale * rng.normal(size=(sc.R_gt.shape[0], 6))).astype(np.float32)


def _dev(ctx, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(ctx.device)


@pytest.mark.parametrize("name", ["tiny", "medium"])
def test_loss_grad_parity(name):
    from paper_2505_04612_amd import api
    ctx = _ctx()
    sc = helpers.scene(name)
    inp = synth.rotation_inputs(sc)
    s = _graph_scene(ctx, sc.R_gt.shape[0], sc.pairs)
    Q = inp.R_rel.reshape(-1, 9).astype(np.float32)
    th = _perturbed(sc, 3)
    loss, grad = api.rotation_loss_grad(s, _dev(ctx, Q), _dev(ctx, th))
    L, g = ra.loss_grad(_f32(th), sc.pairs, _f32(Q).reshape(-1, 3, 3))
    assert abs(loss.item() - L) <= 1e-10 * L
    # float32 records (the tangent part of dL/dR), float64 sums and adjoint
    np.testing.assert_allclose(grad.cpu().numpy(), g, rtol=1e-5, atol=2e-6 * np.abs(g).max())


def _solve_gpu(ctx, s, Q32, th32, K, lr, frac, trace=False, blocks=0):
    from paper_2505_04612_amd import api
    p = _dev(ctx, th32).contiguous()
    m, v = torch.zeros_like(p), torch.zeros_like(p)
    tr = torch.empty(K, dtype=torch.float64, device=ctx.device) if trace else None
    api.rotation_solve(s, _dev(ctx, Q32), p, m, v, K, lr, frac, loss_trace=tr, blocks=blocks)
    assert s.barrier_failures() == 0
    return p.cpu().numpy(), (tr.cpu().numpy() if trace else None)


def test_fused_steps_match_oracle_adam():
    ctx = _ctx()
    sc = helpers.scene("medium")
    inp = synth.rotation_inputs(sc)
    s = _graph_scene(ctx, sc.R_gt.shape[0], sc.pairs)
    Q = inp.R_rel.reshape(-1, 9).astype(np.float32)
    th = _perturbed(sc, 4)
    K, lr, frac = 5, 1e-2, 1e-2
    got, trace = _solve_gpu(ctx, s, Q, th, K, lr, frac, trace=True)
    want, wtr = ra.solve(_f32(th), sc.pairs, _f32(Q).reshape(-1, 3, 3), K, lr, frac)
    # five Adam steps of at most lr each; float32 parameters and moments
    np.testing.assert_allclose(got, want, rtol=0, atol=2e-5)
    # the first loss is at the same stored parameters; later ones at float32
    # parameters against the oracle's float64 ones
    assert abs(trace[0] - wtr[0]) <= 1e-10 * wtr[0]
    np.testing.assert_allclose(trace, wtr, rtol=1e-6)


def test_fused_solve_grid_invariance():
    ctx = _ctx()
    sc = helpers.scene("tiny")
    inp = synth.rotation_inputs(sc)
    s = _graph_scene(ctx, sc.R_gt.shape[0], sc.pairs)
    Q = inp.R_rel.reshape(-1, 9).astype(np.float32)
    th = _perturbed(sc, 5)
    ref, _ = _solve_gpu(ctx, s, Q, th, 60, 1e-2, 1e-2, blocks=1)
    for b in (2, 3, 16):
        got, _ = _solve_gpu(ctx, s, Q, th, 60, 1e-2, 1e-2, blocks=b)
        assert np.array_equal(got, ref), b


@pytest.mark.parametrize("K", [60, 59])
def test_camera_loop_matches_pair_loop(K):
    """The automatic grid runs the loop camera by camera (every pair evaluated
    from both of its cameras, one grid barrier per iteration); a forced
    workgroup count runs it pair by pair.  Both sum the same float32 records
    in float64, in different orders, so they agree to rounding; the camera
    loop is deterministic.  An odd K ends in the second parameter buffer."""
    ctx = _ctx()
    sc = helpers.scene("medium")
    inp = synth.rotation_inputs(sc)
    s = _graph_scene(ctx, sc.R_gt.shape[0], sc.pairs)
    Q = inp.R_rel.reshape(-1, 9).astype(np.float32)
    th = _perturbed(sc, 6)
    a, ta_ = _solve_gpu(ctx, s, Q, th, K, 1e-2, 1e-2, trace=True)
    b, tb = _solve_gpu(ctx, s, Q, th, K, 1e-2, 1e-2, trace=True)
    c, tc = _solve_gpu(ctx, s, Q, th, K, 1e-2, 1e-2, trace=True, blocks=16)
    assert np.array_equal(a, b) and np.array_equal(ta_, tb)
    np.testing.assert_allclose(a, c, rtol=0, atol=1e-5)
    np.testing.assert_allclose(ta_, tc, rtol=1e-9)


@pytest.mark.parametrize("name", ["tiny", "medium"])
def test_solve_endpoint_from_the_oracle_initialisation(name):
    ctx = _ctx()
    sc = helpers.scene(name)
    inp = synth.rotation_inputs(sc)
    N = sc.R_gt.shape[0]
    s = _graph_scene(ctx, N, sc.pairs)
    Q = inp.R_rel.reshape(-1, 9).astype(np.float32)
    R0, _ = ra.initialise(sc.pairs, _f32(Q).reshape(-1, 3, 3), N)
    th0 = _params(R0).astype(np.float32)
    got, trace = _solve_gpu(ctx, s, Q, th0, 500, 1e-2, 1e-2, trace=True)
    want, wtr = ra.solve(_f32(th0), sc.pairs, _f32(Q).reshape(-1, 3, 3), 500, 1e-2, 1e-2)
    # the same L1-type minimum up to the last steps' jitter: the final rate
    # lr0/100 = 1e-4 rad moves a camera by up to 0.006 deg per step and a
    # pair's relative rotation by twice that, more on weakly held cameras;
    # the bar is half the 0.1 deg pose bar of the epipolar solve
    e = ra.relative_rotation_errors(ra.rotations(_f32(got)), ra.rotations(want), sc.pairs)
    assert e.max() < 0.05 and np.median(e) < 0.005, (e.max(), np.median(e))
    assert abs(trace[-1] - wtr[-1]) <= 1e-4 * wtr[-1]
    # and it improves on the initialisation against the truth
    e_gt = ra.relative_rotation_errors(ra.rotations(_f32(got)), sc.R_gt, sc.pairs)
    e_0 = ra.relative_rotation_errors(R0, sc.R_gt, sc.pairs)
    assert np.median(e_gt) < 0.25 * np.median(e_0)


def test_empty_graph():
    from paper_2505_04612_amd import api
    ctx = _ctx()
    s = _graph_scene(ctx, 4, np.zeros((0, 2), np.int32))
    Q = torch.zeros((0, 9), dtype=torch.float32, device=ctx.device)
    th = torch.from_numpy(_params(np.broadcast_to(np.eye(3), (4, 3, 3)).copy()).astype(np.float32)).to(ctx.device)
    loss, grad = api.rotation_loss_grad(s, Q, th)
    assert loss.item() == 0.0 and np.all(grad.cpu().numpy() == 0.0)
    before = th.clone()
    api.rotation_solve(s, Q, th, torch.zeros_like(th), torch.zeros_like(th), 10, 1e-2, 1e-2)
    assert torch.equal(before, th)
    assert s.barrier_failures() == 0


def _init_gpu(ctx, s, Q32, N, steps, seed=0):
    from paper_2505_04612_amd import api
    start = np.random.default_rng(seed).normal(size=(2, 3 * N))
    p, info = api.rotation_init(s, _dev(ctx, Q32), _dev(ctx, start), steps)
    assert s.barrier_failures() == 0
    return p.cpu().numpy(), info.cpu().numpy()


@pytest.mark.parametrize("name,steps", [("tiny", 300), ("medium", 300), ("medium", 150)])
def test_initialisation_parity(name, steps):
    ctx = _ctx()
    sc = helpers.scene(name)
    inp = synth.rotation_inputs(sc)
    N = sc.R_gt.shape[0]
    s = _graph_scene(ctx, N, sc.pairs)
    Q = inp.R_rel.reshape(-1, 9).astype(np.float32)
    got, info = _init_gpu(ctx, s, Q, N, steps)
    R_or, oinfo = ra.initialise(sc.pairs, _f32(Q).reshape(-1, 3, 3), N)
    # both problems' smallest eigenvalues (tiny: 3N = 60 steps span the space)
    w1 = np.linalg.eigvalsh(oinfo["A"])[0]
    w2 = np.linalg.eigvalsh(oinfo["B"])[0]
    assert abs(info[0] - w1) <= 1e-10 * w1 and abs(info[2] - w2) <= 1e-8 * w2, (info, w1, w2)
    # Lanczos stops once its residual bound is below 1e-11 of |T|
    assert 1 <= info[1] <= min(steps, 3 * N)
    # the rotations, up to the sign of each eigenvector (a global rotation):
    # float32 parameters, so ~1e-7 rad, plus the arccos floor of the metric
    e = ra.relative_rotation_errors(ra.rotations(_f32(got)), R_or, sc.pairs)
    assert e.max() < 1e-3, e.max()


def test_initialisation_noise_free_is_exact():
    ctx = _ctx()
    sc = helpers.scene("tiny")
    inp = synth.rotation_inputs(sc, sigma_deg=0.0, outlier_frac=0.0)
    N = sc.R_gt.shape[0]
    s = _graph_scene(ctx, N, sc.pairs)
    got, info = _init_gpu(ctx, s, inp.R_rel.reshape(-1, 9).astype(np.float32), N, 300)
    # the minimiser is any vector of the three-dimensional null space: each
    # gives the truth up to a global rotation
    assert abs(info[0]) < 1e-6
    e = ra.relative_rotation_errors(ra.rotations(_f32(got)), sc.R_gt, sc.pairs)
    assert e.max() < 1e-3, e.max()


def test_whole_stage_initialise_then_solve():
    from paper_2505_04612_amd import api
    ctx = _ctx()
    sc = helpers.scene("medium")
    inp = synth.rotation_inputs(sc)
    N = sc.R_gt.shape[0]
    s = _graph_scene(ctx, N, sc.pairs)
    Q = inp.R_rel.reshape(-1, 9).astype(np.float32)
    p0, _ = _init_gpu(ctx, s, Q, N, 300)
    got, _ = _solve_gpu(ctx, s, Q, p0, 500, 1e-2, 1e-2)
    R0, _ = ra.initialise(sc.pairs, _f32(Q).reshape(-1, 3, 3), N)
    want, _ = ra.solve(_params(R0), sc.pairs, _f32(Q).reshape(-1, 3, 3), 500, 1e-2, 1e-2)
    e = ra.relative_rotation_errors(ra.rotations(_f32(got)), ra.rotations(want), sc.pairs)
    assert e.max() < 0.05 and np.median(e) < 0.005, (e.max(), np.median(e))


def test_initialisation_rejects_an_empty_graph():
    from paper_2505_04612_amd import api
    from paper_2505_04612_amd._lib import FastMapError
    ctx = _ctx()
    s = _graph_scene(ctx, 3, np.zeros((0, 2), np.int32))
    with pytest.raises(FastMapError):
        api.rotation_init(s, torch.zeros((0, 9), dtype=torch.float32, device=ctx.device),
                          torch.ones((2, 9), dtype=torch.float64, device=ctx.device))
