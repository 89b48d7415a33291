"""Check mode of the C ABI (fm_set_check / fm_check): every condition is
forced from the host on a small scene (a NaN coordinate, two cameras at the
same pose, NaN parameters, a NaN Gram entry), so every kernel runs to its
normal end and only reports through the device flag."""
import numpy as np
import pytest
import torch

from paper_2505_04612_amd import _lib, api, solver
from paper_2505_04612_amd._lib import FastMapError

from tests.helpers import scene

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def _scene(ctx, sc, uv=None, dtype=torch.float32):
    return api.Scene.from_numpy(ctx, sc.num_cams, sc.pairs, sc.offsets, sc.uv if uv is None else uv, dtype)


def _params(sc):
    th = np.concatenate([sc.R_init[:, :, 0], sc.R_init[:, :, 1], sc.t_init], axis=1).astype(np.float32)
    return th


def _expect(ctx, bits):
    with pytest.raises(FastMapError) as e:
        ctx.check()
    assert e.value.status == _lib.FM_EDEVICE_CHECK
    assert e.value.flags & bits == bits, (e.value.flags, bits)
    return e.value


def test_clean_data_raises_nothing(ctx):
    sc = scene("tiny")
    s = _scene(ctx, sc)
    ctx.set_check(True)
    try:
        p = torch.from_numpy(_params(sc)).to(ctx.device)
        W, _, Z = api.reweight_build(s, p, 1e-4, 0.1)
        api.epipolar_loss_grad(s, W, p, Z=Z)
        solver.solve(s, p, solver.Schedule(iters=20, round_len=10))
        assert ctx.check() == 0
    finally:
        ctx.set_check(False)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_non_finite_coordinate_is_flagged(ctx, dtype):
    sc = scene("tiny")
    uv = sc.uv.copy()
    uv[sc.num_matches // 2, 3] = np.nan
    s = _scene(ctx, sc, uv, dtype)
    p = torch.from_numpy(_params(sc)).to(ctx.device)
    # off: nothing is reported
    api.reweight_build(s, p, 1e-4, 0.1)
    assert ctx.check() == 0
    ctx.set_check(True)
    try:
        api.build_pair_grams(s)
        err = _expect(ctx, _lib.FM_CHECK_COORDS)
        assert "non-finite match coordinates" in str(err)
        # the flag was cleared by the read
        assert ctx.check() == 0
        api.reweight_build(s, p, 1e-4, 0.1)
        _expect(ctx, _lib.FM_CHECK_COORDS)
    finally:
        ctx.set_check(False)


def test_degenerate_pair_is_flagged_and_adds_nothing(ctx):
    """Two cameras at the same pose with the identity rotation (exact through
    Gram-Schmidt, so R_ij = I and t_ij = t_j - t_i = 0 exactly): E_n has no
    direction.  The pair adds 0 to the loss and its residuals are 0 (kept with
    weight 1/delta at any threshold), and check mode reports it at those
    poses."""
    sc = scene("tiny")
    s = _scene(ctx, sc)
    th = _params(sc)
    i, j = (int(x) for x in sc.pairs[0])
    th[i, :6] = th[j, :6] = [1, 0, 0, 0, 1, 0]
    th[j, 6:] = th[i, 6:]
    p = torch.from_numpy(th).to(ctx.device)
    W, _ = api.build_pair_grams(s, f64=True, f32=False)
    ctx.set_check(True)
    try:
        loss, grad = api.epipolar_loss_grad(s, W, p, inv_Z=1.0)
        flags = _expect(ctx, _lib.FM_CHECK_DEGENERATE).flags
        assert not flags & (_lib.FM_CHECK_PARAMS | _lib.FM_CHECK_LOSS)
        w, r, _ = api.reweight(s, p, 1e-4, 0.1, residuals=True)
        _expect(ctx, _lib.FM_CHECK_DEGENERATE)
    finally:
        ctx.set_check(False)
    lo, hi = int(sc.offsets[0]), int(sc.offsets[1])
    assert torch.all(r[lo:hi] == 0)
    # omega = 1/max(0, delta) (the kernel's float32 reciprocal)
    assert np.allclose(w[lo:hi].cpu().numpy(), 1.0 / np.float32(1e-4), rtol=1e-6)
    # the pair's share of the loss is 0: the loss equals the loss with the
    # pair's Gram zeroed
    W0 = W.clone()
    W0[0] = 0
    l0, _ = api.epipolar_loss_grad(s, W0, p, inv_Z=1.0)
    assert float(loss.item()) == float(l0.item())
    assert torch.all(torch.isfinite(grad))


def test_nearly_coincident_cameras_are_flagged(ctx):
    """Two cameras at the same float32 pose with a general rotation: R_ij is
    the identity only to float64 rounding, so t_ij is ~1e-16 of t and its
    direction is noise; check mode reports it."""
    sc = scene("tiny")
    s = _scene(ctx, sc)
    th = _params(sc)
    i, j = (int(x) for x in sc.pairs[3])
    th[j] = th[i]
    p = torch.from_numpy(th).to(ctx.device)
    ctx.set_check(True)
    try:
        api.reweight_build(s, p, 1e-4, 0.1)
        _expect(ctx, _lib.FM_CHECK_DEGENERATE)
    finally:
        ctx.set_check(False)


def test_non_finite_parameters_are_flagged(ctx):
    sc = scene("tiny")
    s = _scene(ctx, sc)
    th = _params(sc)
    th[3, 7] = np.inf
    p = torch.from_numpy(th).to(ctx.device)
    ctx.set_check(True)
    try:
        api.reweight_build(s, p, 1e-4, 0.1)
        _expect(ctx, _lib.FM_CHECK_PARAMS)
    finally:
        ctx.set_check(False)


def test_non_finite_loss_is_flagged_by_loss_and_solve(ctx):
    """A NaN planted in one pair's Gram makes the loss NaN: the standalone
    loss call and the fused solve (loss trace, then the parameters it moved)
    both report it."""
    sc = scene("tiny")
    s = _scene(ctx, sc)
    p = torch.from_numpy(_params(sc)).to(ctx.device)
    W, _ = api.build_pair_grams(s, f64=True, f32=False)
    W[5, 7] = float("nan")
    ctx.set_check(True)
    try:
        loss, _ = api.epipolar_loss_grad(s, W, p, inv_Z=1e-5)
        assert not bool(torch.isfinite(loss).item())
        _expect(ctx, _lib.FM_CHECK_LOSS)
        m, v = torch.zeros_like(p), torch.zeros_like(p)
        trace = torch.empty(3, dtype=torch.float64, device=ctx.device)
        api.epipolar_solve(s, W, p, m, v, 3, 3e-3, 1e-2, 1e-3, 0, 3, inv_Z=1e-5, loss_trace=trace)
        _expect(ctx, _lib.FM_CHECK_LOSS | _lib.FM_CHECK_PARAMS)
    finally:
        ctx.set_check(False)
