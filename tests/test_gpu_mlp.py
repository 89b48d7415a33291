"""Learned-weight form: GPU features and MLP forward/backward against the FP64
oracle (oracle/mlp.py).

Tolerances: the 64x64 layer uses float16 operands (unit roundoff 4.9e-4) with
float32 accumulation, so outputs are compared with an absolute 2e-3 (outputs
lie in [0, 1]) and gradients normwise within 2e-2; features are float32
conversions of float64 values (relative 1e-6, parallax absolute 1e-6 rad).
"""
import numpy as np
import pytest
import torch

from oracle import ea, mlp
from tests.helpers import scene, stored

pytestmark = pytest.mark.gpu


def _weights(seed):
    p = mlp.init_params(seed)
    rng = np.random.default_rng(seed + 1)
    for k in p:
        p[k] = p[k] + rng.normal(0.0, 0.05, p[k].shape)
    return p


@pytest.mark.parametrize("M", [1, 15, 16, 17, 1000, 40_001])
def test_mlp_forward_backward_parity(M):
    from paper_2505_04612_amd import api
    ctx = api.default_context()
    rng = np.random.default_rng(M)
    feats = (rng.normal(size=(M, 3)) * [2.0, 1.0, 0.1] + [-6.0, 5.0, 0.2]).astype(np.float32)
    mean, std = np.array([-6.0, 5.0, 0.2]), np.array([2.0, 1.0, 0.1])
    p = _weights(M % 7)
    w = api.MlpWeights(ctx.device)
    w.load_numpy(p, mean, std)
    f = torch.from_numpy(feats).to(ctx.device)
    out, act = api.mlp_forward(ctx, w, f, keep_act=True)
    out2, _ = api.mlp_forward(ctx, w, f, out_scale=3.0)
    ref, _ = mlp.forward({k: v.astype(np.float32).astype(np.float64) for k, v in p.items()},
                         feats.astype(np.float64), mean.astype(np.float32), std.astype(np.float32))
    o = out.cpu().numpy()
    assert np.abs(o - ref).max() <= 2e-3
    assert np.allclose(out2.cpu().numpy(), 3.0 * o, rtol=1e-6)
    dout = rng.normal(size=M).astype(np.float32)
    g = api.mlp_backward(ctx, w, f, act, torch.from_numpy(dout).to(ctx.device))
    g2 = api.mlp_backward(ctx, w, f, act, torch.from_numpy(dout).to(ctx.device))
    assert torch.equal(g.flat, g2.flat), "MLP backward is not deterministic"
    gref = mlp.backward({k: v.astype(np.float32).astype(np.float64) for k, v in p.items()},
                        feats.astype(np.float64), mean.astype(np.float32), std.astype(np.float32),
                        dout.astype(np.float64))
    gg = g.to_numpy()
    for k in mlp.SHAPES:
        err = np.linalg.norm(gg[k] - gref[k])
        assert err <= 2e-2 * np.linalg.norm(gref[k]) + 1e-4 * np.sqrt(M), (k, err, np.linalg.norm(gref[k]))


def test_mlp_forward_parity_many_tiles():
    """200,003 matches: more 16-match tiles than the forward grid's
    wavefronts, so each wavefront takes several tiles, with a ragged last
    tile.  The backward over this many matches is checked at a looser bound:
    its gradient error grows with M (FP16 operands in its products over the
    matches; 2.2 % of the norm for b2 here)."""
    from paper_2505_04612_amd import api
    ctx = api.default_context()
    M = 200_003
    rng = np.random.default_rng(M)
    feats = (rng.normal(size=(M, 3)) * [2.0, 1.0, 0.1] + [-6.0, 5.0, 0.2]).astype(np.float32)
    mean, std = np.array([-6.0, 5.0, 0.2]), np.array([2.0, 1.0, 0.1])
    p = _weights(3)
    w = api.MlpWeights(ctx.device)
    w.load_numpy(p, mean, std)
    f = torch.from_numpy(feats).to(ctx.device)
    out, act = api.mlp_forward(ctx, w, f, keep_act=True)
    out_plain, _ = api.mlp_forward(ctx, w, f)
    ref, _ = mlp.forward({k: v.astype(np.float32).astype(np.float64) for k, v in p.items()},
                         feats.astype(np.float64), mean.astype(np.float32), std.astype(np.float32))
    o = out.cpu().numpy()
    assert np.abs(o - ref).max() <= 2e-3
    assert torch.equal(out, out_plain)
    dout = rng.normal(size=M).astype(np.float32)
    g = api.mlp_backward(ctx, w, f, act, torch.from_numpy(dout).to(ctx.device))
    gref = mlp.backward({k: v.astype(np.float32).astype(np.float64) for k, v in p.items()},
                        feats.astype(np.float64), mean.astype(np.float32), std.astype(np.float32),
                        dout.astype(np.float64))
    gg = g.to_numpy()
    for k in mlp.SHAPES:
        err = np.linalg.norm(gg[k] - gref[k])
        assert err <= 4e-2 * np.linalg.norm(gref[k]) + 1e-4 * np.sqrt(M), (k, err, np.linalg.norm(gref[k]))


@pytest.mark.parametrize("name,dtype", [("tiny", torch.float64), ("medium", torch.float32)])
def test_match_features_parity(name, dtype):
    from paper_2505_04612_amd import api
    sc = scene(name)
    ctx = api.default_context()
    s = api.Scene.from_numpy(ctx, sc.num_cams, sc.pairs, sc.offsets, sc.uv, dtype)
    th = ea.params_from_poses(sc.R_init, sc.t_init).astype(np.float32)
    f = api.match_features(s, torch.from_numpy(th).to(ctx.device), 1e-4).cpu().numpy()
    ref = mlp.features(th.astype(np.float64), sc.pairs, sc.offsets, stored(sc.uv, dtype), float(np.float32(1e-4)))
    assert np.allclose(f[:, 0], ref[:, 0], rtol=1e-6, atol=1e-5)
    assert np.allclose(f[:, 1], ref[:, 1], rtol=1e-6)
    assert np.allclose(f[:, 2], ref[:, 2], rtol=1e-5, atol=1e-6)
