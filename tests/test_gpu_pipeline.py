"""The pose stages in sequence on the GPU (rotation averaging, grid search,
translation averaging, epipolar adjustment): the layout conversion between
them against the oracle's Gram-Schmidt, and the whole chain on the medium
scene against the truth (each stage has its own parity tests)."""
import numpy as np
import pytest
import torch

from oracle import ea
from paper_2505_04612_amd import synth
from tests import helpers

pytestmark = pytest.mark.gpu


def test_poses_from_centres_parity():
    from paper_2505_04612_amd import api
    ctx = api.default_context()
    rng = np.random.default_rng(31)
    N = 1000
    p6 = rng.normal(size=(N, 6)).astype(np.float32)
    o = rng.normal(size=(N, 3)).astype(np.float32)
    got = api.poses_from_centres(ctx, torch.from_numpy(p6).to(ctx.device), torch.from_numpy(o).to(ctx.device))
    got = got.cpu().numpy()
    R = ea.rot_from_6d(p6[:, 0:3].astype(np.float64), p6[:, 3:6].astype(np.float64))
    np.testing.assert_array_equal(got[:, 0:6], p6)
    np.testing.assert_allclose(got[:, 6:9], -np.einsum("nab,nb->na", R, o.astype(np.float64)), rtol=0, atol=2e-6)


def test_whole_pose_pipeline_on_the_medium_scene():
    from paper_2505_04612_amd import api, pipeline
    ctx = api.default_context()
    sc = helpers.scene("medium")
    dev = ctx.device
    s = api.Scene.from_numpy(ctx, sc.num_cams, sc.pairs, sc.offsets, sc.uv, torch.float32)
    rin = synth.rotation_inputs(sc)
    o = -np.einsum("nba,nb->na", sc.R_gt, sc.t_gt)
    i, j = sc.pairs[:, 0], sc.pairs[:, 1]
    prior = np.einsum("pab,pb->pa", sc.R_gt[j], o[i] - o[j])
    prior /= np.linalg.norm(prior, axis=1, keepdims=True)
    keep = torch.from_numpy((~sc.outlier).astype(np.float32)).to(dev)
    params, stages = pipeline.run(s, torch.from_numpy(rin.R_rel.reshape(-1, 9).astype(np.float32)).to(dev),
                                  torch.from_numpy(prior.astype(np.float32)).to(dev), keep)
    assert s.barrier_failures() == 0
    gt = np.concatenate([sc.R_gt[:, :, 0], sc.R_gt[:, :, 1], sc.t_gt], 1)
    rot0, tra0 = ea.relative_pose_errors(stages["averaged"].cpu().numpy().astype(np.float64), gt, sc.pairs)
    rot, tra = ea.relative_pose_errors(params.cpu().numpy().astype(np.float64), gt, sc.pairs)
    # the averaging stages land close enough for epipolar adjustment, which
    # then improves both rotations and translation directions
    assert np.median(rot0) < 0.5 and np.median(tra0) < 1.0, (np.median(rot0), np.median(tra0))
    assert np.median(rot) < 0.25 and np.median(tra) < 0.2, (np.median(rot), np.median(tra))
    assert np.median(rot) < np.median(rot0) and np.median(tra) < np.median(tra0)
    assert rot.max() < 2.0
