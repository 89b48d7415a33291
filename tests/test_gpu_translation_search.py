"""Relative-translation grid search on the GPU (appendix on global
translation, "Relative Translation") against the FP64 oracle on the same
Grams, rotations, candidates and priors."""
import numpy as np
import pytest
import torch

from oracle import grid_search as gs
from tests import helpers

pytestmark = pytest.mark.gpu


def _ctx():
    from paper_2505_04612_amd import api
    return api.default_context()


def _dev(ctx, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(ctx.device)


def _check(got_t, got_best, got_err, W, counts, Rij, cand, prior):
    want_t, want_best, err = gs.grid_search(W, counts, Rij, cand, prior)
    live = counts > 0
    srt = np.sort(err, axis=1)
    clear = live & ((srt[:, 1] - srt[:, 0]) > 1e-9 * np.maximum(np.abs(srt[:, 0]), 1e-300))
    # the winner wherever the two best errors differ by more than rounding,
    # a minimal candidate everywhere
    assert np.array_equal(got_best[clear], want_best[clear])
    idx = np.where(live)[0]
    assert np.all(err[idx, got_best[idx]] <= srt[idx, 0] + 1e-9 * np.abs(srt[idx, 0]) + 1e-300)
    assert np.all(got_best[~live] == -1)
    np.testing.assert_allclose(got_err[live], srt[live, 0], rtol=1e-9, atol=1e-300)
    # the output is the winning candidate with the prior's sign, in float32
    sgn = np.where(np.sum(cand[np.maximum(got_best, 0)] * prior, axis=1) < 0, -1.0, 1.0)
    want = np.where(live[:, None], sgn[:, None] * cand[np.maximum(got_best, 0)], prior)
    np.testing.assert_array_equal(got_t, want.astype(np.float32))


@pytest.mark.parametrize("name,C", [("tiny", 3000), ("medium", 5000)])
def test_search_parity(name, C):
    from paper_2505_04612_amd import api
    ctx = _ctx()
    sc = helpers.scene(name)
    dt = torch.float64 if name == "tiny" else torch.float32
    s = api.Scene.from_numpy(ctx, sc.num_cams, sc.pairs, sc.offsets, sc.uv, dt)
    W64, _ = api.build_pair_grams(s, f32=False)
    params = np.concatenate([sc.R_gt[:, :, 0], sc.R_gt[:, :, 1], sc.t_gt], 1).astype(np.float32)
    o = -np.einsum("nba,nb->na", sc.R_gt, sc.t_gt)
    i, j = sc.pairs[:, 0], sc.pairs[:, 1]
    prior = np.einsum("pab,pb->pa", sc.R_gt[j], o[i] - o[j])
    prior = (prior / np.linalg.norm(prior, axis=1, keepdims=True)).astype(np.float32)
    cand = gs.fibonacci_sphere(C)
    t, best, err = api.translation_search(s, W64, _dev(ctx, params), _dev(ctx, cand), _dev(ctx, prior))
    W = helpers.expand36(W64.cpu().numpy())
    Rij = gs.relative_rotations(params.astype(np.float64), sc.pairs)
    _check(t.cpu().numpy(), best.cpu().numpy(), err.cpu().numpy(), W, np.diff(sc.offsets), Rij, cand,
           prior.astype(np.float64))
    # the library's lattice is the oracle's
    np.testing.assert_allclose(api.fibonacci_sphere(C, ctx.device).cpu().numpy(), cand, atol=1e-15)


def test_search_parity_on_a_large_graph_of_arbitrary_forms():
    from paper_2505_04612_amd import api
    ctx = _ctx()
    rng = np.random.default_rng(21)
    N, P = 300, 20_001
    a = rng.integers(0, N, size=P)
    b = (a + 1 + rng.integers(0, N - 1, size=P)) % N
    pairs = np.stack([np.minimum(a, b), np.maximum(a, b)], 1).astype(np.int32)
    counts = rng.integers(0, 5, size=P)
    offsets = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    uv = rng.uniform(-0.5, 0.5, size=(int(offsets[-1]), 4))
    s = api.Scene.from_numpy(ctx, N, pairs, offsets, uv, torch.float32)
    W36 = rng.normal(size=(P, 36))
    th = rng.normal(size=(N, 9)).astype(np.float32)
    prior = rng.normal(size=(P, 3)).astype(np.float32)
    cand = gs.fibonacci_sphere(777)
    t, best, err = api.translation_search(s, _dev(ctx, W36), _dev(ctx, th), _dev(ctx, cand), _dev(ctx, prior))
    Rij = gs.relative_rotations(th.astype(np.float64), pairs)
    _check(t.cpu().numpy(), best.cpu().numpy(), err.cpu().numpy(), helpers.expand36(W36), counts, Rij, cand,
           prior.astype(np.float64))


def test_single_candidate_and_empty_pairs():
    from paper_2505_04612_amd import api
    ctx = _ctx()
    pairs = np.array([[0, 1], [1, 2], [0, 2]], np.int32)
    s = api.Scene.from_numpy(ctx, 3, pairs, np.zeros(4, np.int64), np.zeros((0, 4)), torch.float32)
    prior = np.array([[0, 0, 1], [0, 1, 0], [1, 0, 0]], np.float32)
    params = np.tile(np.array([1, 0, 0, 0, 1, 0, 0, 0, 0], np.float32), (3, 1))
    t, best, err = api.translation_search(s, torch.zeros((3, 36), dtype=torch.float64, device=ctx.device),
                                          _dev(ctx, params), _dev(ctx, np.array([[1.0, 0.0, 0.0]])),
                                          _dev(ctx, prior))
    np.testing.assert_array_equal(t.cpu().numpy(), prior)
    assert np.all(best.cpu().numpy() == -1)
