"""Pins of the FP64 focal-refinement oracle (Sec. 3.3: focal lengths built
into the essential matrices, which become fundamental matrices) against what
the mathematics fixes and against the pinned epipolar oracle."""
import numpy as np
import pytest

from oracle import ea
from oracle import focal as fo
from paper_2505_04612_amd import synth

KAPPA = 1.1   # coordinates normalised with a focal 1/1.1 of the true one


@pytest.fixture(scope="module")
def tiny():
    return synth.tiny()


@pytest.fixture(scope="module")
def clean():
    return synth.noise_free(synth.tiny)


def _theta(sc):
    return np.concatenate([sc.R_gt[:, :, 0], sc.R_gt[:, :, 1], sc.t_gt], 1)


def test_unit_scales_give_half_the_epipolar_loss_and_gradient(tiny):
    # |[t_hat]_x R|_F^2 = 2 for any pose, so at phi = 0 the normalised loss is
    # exactly half the epipolar one and its pose gradient half the epipolar
    # gradient (the normalisation's own derivative is orthogonal to e)
    W = ea.pair_grams(tiny.uv, tiny.offsets)
    theta = np.concatenate([tiny.R_init[:, :, 0], tiny.R_init[:, :, 1], tiny.t_init], 1)
    phi = np.zeros(len(theta))
    inv_Z = 1.0 / tiny.num_matches
    L, g, gp = fo.loss_grad(theta, phi, tiny.pairs, W, inv_Z)
    Le, ge = ea.loss_grad(theta, tiny.pairs, W, inv_Z)
    assert L == pytest.approx(Le / 2, rel=1e-12)
    np.testing.assert_allclose(g, ge / 2, rtol=1e-9, atol=1e-12 * np.abs(ge).max())
    assert L == pytest.approx(fo.loss(theta, phi, tiny.pairs, W, inv_Z), rel=1e-13)


def test_central_differences(tiny):
    W = ea.pair_grams(tiny.uv, tiny.offsets)
    rng = np.random.default_rng(5)
    theta = np.concatenate([tiny.R_init[:, :, 0], tiny.R_init[:, :, 1], tiny.t_init], 1)
    phi = 0.1 * rng.normal(size=len(theta))
    inv_Z = 1.0 / tiny.num_matches
    L, g, gp = fo.loss_grad(theta, phi, tiny.pairs, W, inv_Z)
    h = 1e-6
    for _ in range(6):
        d = rng.normal(size=theta.shape)
        dp = rng.normal(size=phi.shape)
        fd = (fo.loss(theta + h * d, phi + h * dp, tiny.pairs, W, inv_Z)
              - fo.loss(theta - h * d, phi - h * dp, tiny.pairs, W, inv_Z)) / (2 * h)
        an = (g * d).sum() + (gp * dp).sum()
        assert abs(fd - an) <= 1e-7 * max(abs(an), 1e-3 * abs(L)), (fd, an)


def test_loss_vanishes_at_the_true_focal_scale(clean):
    uv = clean.uv * KAPPA
    W = ea.pair_grams(uv, clean.offsets)
    theta = _theta(clean)
    inv_Z = 1.0 / clean.num_matches
    N = len(theta)
    L_true = fo.loss(theta, np.full(N, np.log(KAPPA)), clean.pairs, W, inv_Z)
    L_unit = fo.loss(theta, np.zeros(N), clean.pairs, W, inv_Z)
    assert L_true < 1e-12 * L_unit and L_unit > 0
    # moving all scales together from 1 toward the truth lowers the loss
    # (single cameras couple with their neighbours' poses and scales)
    _, _, gp = fo.loss_grad(theta, np.zeros(N), clean.pairs, W, inv_Z)
    assert gp.sum() < 0


def test_adam_recovers_the_focal_scale(clean):
    uv = clean.uv * KAPPA
    W = ea.pair_grams(uv, clean.offsets)
    theta = _theta(clean)
    N = len(theta)
    iz = 1.0 / clean.num_matches
    # poses held at the truth: the scales go exactly to log(kappa)
    th, ph, trace = fo.solve(theta, np.zeros(N), clean.pairs, W, iz, 400, lr_rot=0.0, lr_t=0.0, lr_phi=1e-2)
    np.testing.assert_allclose(ph, np.log(KAPPA), atol=1e-6)
    # poses free as well: focal and translation share a flat valley, the loss
    # still falls by four orders and the scales stay close to the truth
    th, ph, trace = fo.solve(theta, np.zeros(N), clean.pairs, W, iz, 400, lr_rot=1e-4, lr_t=1e-4, lr_phi=1e-2)
    assert trace[-1] < 1e-4 * trace[0]
    np.testing.assert_allclose(ph, np.log(KAPPA), atol=5e-3)
    # (the poses drift a little along the same valley: 0.15 deg here)
    rot, tra = ea.relative_pose_errors(th, theta, clean.pairs)
    assert rot.max() < 0.5
