"""The camera-by-camera persistent loops on a graph with more cameras than
co-resident wavefronts (5,000 cameras; 256 workgroups of 8 wavefronts at
most), so that wavefronts take several cameras in turn: each loop against
its pair-by-pair form (forced workgroup count) and against itself.  The
two forms sum the same float32 records in float64 in different orders, so
they agree to rounding."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

N_CAMS = 5000


def _ctx():
    from paper_2505_04612_amd import api
    return api.default_context()


def _banded_pairs(N, reach):
    return np.array([(i, i + k) for i in range(N) for k in range(1, reach + 1) if i + k < N], dtype=np.int32)


def _rotations(rng, n):
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    return np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w),
                     2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w),
                     2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)], 1).reshape(n, 3, 3)


def _graph_scene(ctx, N, pairs):
    from paper_2505_04612_amd import api
    P = len(pairs)
    return api.Scene.from_numpy(ctx, N, pairs, np.zeros(P + 1, np.int64), np.zeros((0, 4)), torch.float32)


def test_epipolar_camera_loop_with_strided_cameras():
    from paper_2505_04612_amd import api
    ctx = _ctx()
    rng = np.random.default_rng(11)
    pairs = _banded_pairs(N_CAMS, 3)
    P = len(pairs)
    offsets = (np.arange(P + 1) * 9).astype(np.int64)
    uv = rng.normal(scale=0.5, size=(9 * P, 4)).astype(np.float32)
    s = api.Scene.from_numpy(ctx, N_CAMS, pairs, offsets, uv, torch.float32)
    W64, _ = api.build_pair_grams(s)
    R = _rotations(rng, N_CAMS)
    th = np.concatenate([R[:, :, 0], R[:, :, 1], rng.normal(size=(N_CAMS, 3))], 1).astype(np.float32)
    out = []
    for blocks in (0, 0, 64):
        p = torch.from_numpy(th).to(ctx.device)
        m, v = torch.zeros_like(p), torch.zeros_like(p)
        tr = torch.zeros(20, dtype=torch.float64, device=ctx.device)
        api.epipolar_solve(s, W64, p, m, v, 20, 3e-3, 1e-2, 1e-2, 0, 20, inv_Z=1.0 / (9 * P), blocks=blocks,
                           loss_trace=tr)
        out.append((p, m, v, tr))
    assert s.barrier_failures() == 0
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)
    torch.testing.assert_close(out[0][3], out[2][3], rtol=1e-9, atol=0)
    torch.testing.assert_close(out[0][0], out[2][0], rtol=0, atol=1e-5)


def test_translation_camera_loop_with_strided_cameras():
    from paper_2505_04612_amd import api
    ctx = _ctx()
    rng = np.random.default_rng(12)
    pairs = _banded_pairs(N_CAMS, 3)
    s = _graph_scene(ctx, N_CAMS, pairs)
    d = rng.normal(size=(len(pairs), 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    dirs = torch.from_numpy(d.astype(np.float32)).to(ctx.device)
    cen = rng.normal(size=(3, N_CAMS, 3)).astype(np.float32)
    out = []
    for blocks in (0, 0, 64):
        c = torch.from_numpy(cen).to(ctx.device)
        m, v = torch.zeros_like(c), torch.zeros_like(c)
        tr = torch.zeros((3, 31), dtype=torch.float64, device=ctx.device)
        api.translation_solve(s, dirs, c, m, v, 31, 3e-2, 1e-2, loss_trace=tr, blocks=blocks)
        out.append((c, tr))
    assert s.barrier_failures() == 0
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    torch.testing.assert_close(out[0][1], out[2][1], rtol=1e-6, atol=0)
    torch.testing.assert_close(out[0][0], out[2][0], rtol=0, atol=1e-4)


def test_rotation_camera_loop_with_strided_cameras():
    from paper_2505_04612_amd import api
    ctx = _ctx()
    rng = np.random.default_rng(13)
    pairs = _banded_pairs(N_CAMS, 3)
    s = _graph_scene(ctx, N_CAMS, pairs)
    Q = torch.from_numpy(_rotations(rng, len(pairs)).reshape(-1, 9).astype(np.float32)).to(ctx.device)
    R = _rotations(rng, N_CAMS)
    th = np.concatenate([R[:, :, 0], R[:, :, 1]], 1).astype(np.float32)
    out = []
    for blocks in (0, 0, 64):
        p = torch.from_numpy(th).to(ctx.device)
        m, v = torch.zeros_like(p), torch.zeros_like(p)
        tr = torch.zeros(25, dtype=torch.float64, device=ctx.device)
        api.rotation_solve(s, Q, p, m, v, 25, 1e-2, 1e-2, loss_trace=tr, blocks=blocks)
        out.append((p, tr))
    assert s.barrier_failures() == 0
    assert torch.equal(out[0][0], out[1][0]) and torch.equal(out[0][1], out[1][1])
    torch.testing.assert_close(out[0][1], out[2][1], rtol=1e-9, atol=0)
    torch.testing.assert_close(out[0][0], out[2][0], rtol=0, atol=1e-5)
