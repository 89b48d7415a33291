"""Differentiation form: the hand-written adjoint behind torch.autograd.Function,
checked against FP64 central differences of the oracle on the diffprec
workload (1,000 nadir cameras, ~34k pairs, ~25M BF16-stored matches), along
100 random parameter perturbations.

Tolerance: |g_gpu . d - FD(d)| <= 2e-4 * |g| |d| per direction.  The GPU
gradient is float32 per pair record (relative 6e-8) on a Gram accumulated in
float32 (measured normwise error ~1e-7); the FP64 central difference with
h = 1e-6 carries O(h^2) truncation and ~1e-10 rounding error relative to |g|.
"""
import numpy as np
import pytest
import torch

from oracle import ea
from tests.helpers import scene, stored

pytestmark = pytest.mark.gpu


def test_adjoint_directional_derivatives_diffprec():
    from paper_2505_04612_amd import api
    from paper_2505_04612_amd.autograd import epipolar_loss
    sc = scene("diffprec")
    ctx = api.default_context()
    s = api.Scene.from_numpy(ctx, sc.num_cams, sc.pairs, sc.offsets, sc.uv, torch.bfloat16)
    W64, _ = api.build_pair_grams(s)
    th = ea.params_from_poses(sc.R_init, sc.t_init).astype(np.float32)
    inv_Z = 1.0 / sc.num_matches
    p = torch.from_numpy(th).to(ctx.device).requires_grad_(True)
    L = epipolar_loss(p, s, W64, inv_Z)
    (L * 3.0).backward()
    g = p.grad.detach().cpu().numpy().astype(np.float64) / 3.0
    x = stored(sc.uv, torch.bfloat16)
    W = ea.pair_grams(x, sc.offsets)
    th64 = th.astype(np.float64)
    L_ref, g_ref = ea.loss_grad(th64, sc.pairs, W, inv_Z)
    assert abs(float(L.item()) - L_ref) <= 1e-5 * abs(L_ref)
    rng = np.random.default_rng(100)
    gn = np.linalg.norm(g)
    h = 1e-6
    worst = 0.0
    for _ in range(100):
        d = rng.normal(size=th.shape)
        d /= np.linalg.norm(d)
        fd = (ea.loss_from_grams(th64 + h * d, sc.pairs, W, inv_Z)
              - ea.loss_from_grams(th64 - h * d, sc.pairs, W, inv_Z)) / (2 * h)
        worst = max(worst, abs(float(np.sum(g * d)) - fd) / gn)
    assert worst <= 2e-4, worst
    assert np.linalg.norm(g - g_ref) <= 2e-4 * np.linalg.norm(g_ref)


def test_autograd_function_composes_with_torch():
    """The Function is usable inside a torch computation: a weighted sum of two
    losses differentiates to the weighted sum of the library's gradients."""
    from paper_2505_04612_amd import api
    from paper_2505_04612_amd.autograd import epipolar_loss
    sc = scene("tiny")
    ctx = api.default_context()
    s = api.Scene.from_numpy(ctx, sc.num_cams, sc.pairs, sc.offsets, sc.uv, torch.float64)
    W64, _ = api.build_pair_grams(s)
    th = torch.from_numpy(ea.params_from_poses(sc.R_init, sc.t_init).astype(np.float32)).to(ctx.device)
    p = th.clone().requires_grad_(True)
    loss = 2.0 * epipolar_loss(p, s, W64, 1e-4) + 0.5 * epipolar_loss(p, s, W64, 1e-4)
    loss.backward()
    _, g = api.epipolar_loss_grad(s, W64, th, inv_Z=1e-4)
    assert torch.allclose(p.grad, 2.5 * g, rtol=1e-6, atol=0)
