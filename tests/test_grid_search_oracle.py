"""Pins of the FP64 relative-translation grid-search oracle (appendix on global
translation, "Relative Translation") against what the paper and the
mathematics fix, independent of the oracle's own formulas."""
import numpy as np
import pytest

from oracle import ea
from oracle import grid_search as gs
from paper_2505_04612_amd import synth


@pytest.fixture(scope="module")
def tiny():
    return synth.tiny()


def _gt(sc):
    theta = np.concatenate([sc.R_gt[:, :, 0], sc.R_gt[:, :, 1], sc.t_gt], 1)
    Rij = gs.relative_rotations(theta, sc.pairs)
    o = -np.einsum("nba,nb->na", sc.R_gt, sc.t_gt)
    i, j = sc.pairs[:, 0], sc.pairs[:, 1]
    t = np.einsum("pab,pb->pa", sc.R_gt[j], o[i] - o[j])
    return theta, Rij, t / np.linalg.norm(t, axis=1, keepdims=True)


def test_errors_are_the_mean_squared_epipolar_error_of_the_matches(tiny):
    theta, Rij, t_true = _gt(tiny)
    W = ea.pair_grams(tiny.uv, tiny.offsets)
    counts = np.diff(tiny.offsets)
    rng = np.random.default_rng(1)
    cand = rng.normal(size=(5, 3))
    cand /= np.linalg.norm(cand, axis=1, keepdims=True)
    err = gs.candidate_errors(W, counts, Rij, cand)
    for n in (0, 7, 100):
        lo, hi = tiny.offsets[n], tiny.offsets[n + 1]
        for c in range(5):
            t = cand[c]
            T = np.array([[0.0, -t[2], t[1]], [t[2], 0.0, -t[0]], [-t[1], t[0], 0.0]])
            F = T @ Rij[n]
            brute = 0.0
            for m in range(lo, hi):
                x1 = np.array([tiny.uv[m, 0], tiny.uv[m, 1], 1.0])
                x2 = np.array([tiny.uv[m, 2], tiny.uv[m, 3], 1.0])
                brute += float(x2 @ F @ x1) ** 2
            assert err[n, c] == pytest.approx(brute / (hi - lo), rel=1e-10)


def test_three_by_three_form_matches_the_candidate_errors(tiny):
    theta, Rij, _ = _gt(tiny)
    W = ea.pair_grams(tiny.uv, tiny.offsets)
    counts = np.diff(tiny.offsets)
    A = gs.translation_forms(W, Rij)
    rng = np.random.default_rng(2)
    t = rng.normal(size=(4, 3))
    err = gs.candidate_errors(W, counts, Rij, t)
    q = np.einsum("ca,pab,cb->pc", t, A, t) / counts[:, None]
    np.testing.assert_allclose(q, err, rtol=1e-10)
    np.testing.assert_allclose(A, np.swapaxes(A, -1, -2), atol=1e-12 * np.abs(A).max())


def test_noise_free_truth_wins_and_keeps_the_prior_sign(tiny):
    clean = synth.noise_free(synth.tiny)
    theta, Rij, t_true = _gt(clean)
    W = ea.pair_grams(clean.uv, clean.offsets)
    counts = np.diff(clean.offsets)
    cand = np.concatenate([gs.fibonacci_sphere(500), t_true[:3]])   # the truth of pairs 0..2 among them
    t, best, err = gs.grid_search(W, counts, Rij, cand, t_true)
    for n in range(3):
        assert best[n] == 500 + n
        np.testing.assert_allclose(t[n], t_true[n], atol=1e-15)
        assert err[n, 500 + n] < 1e-12 * err[n].max()      # the FP64 cancellation floor
    # the error is even: with the opposite prior the opposite vector is returned
    t2, _, _ = gs.grid_search(W, counts, Rij, cand, -t_true)
    np.testing.assert_allclose(t2[:3], -t_true[:3], atol=1e-15)


def test_winner_is_within_the_lattice_spacing_of_the_form_minimiser(tiny):
    theta, Rij, t_true = _gt(tiny)
    W = ea.pair_grams(tiny.uv, tiny.offsets)
    counts = np.diff(tiny.offsets)
    C = 4000
    cand = gs.fibonacci_sphere(C)
    t, best, err = gs.grid_search(W, counts, Rij, cand, t_true)
    A = gs.translation_forms(W, Rij)
    _, V = np.linalg.eigh(A)
    v = V[:, :, 0]
    ang = np.degrees(np.arccos(np.clip(np.abs(np.sum(t * v, axis=1)), 0, 1)))
    # covering radius of the lattice (largest distance to the nearest point)
    probe = np.random.default_rng(3).normal(size=(20000, 3))
    probe /= np.linalg.norm(probe, axis=1, keepdims=True)
    cover = np.degrees(np.arccos(np.max(probe @ cand.T, axis=1))).max()
    # the minimum of a quadratic form on the sphere sits at its smallest
    # eigenvector; a lattice point within the covering radius of it has an
    # error within (cover angle)^2 * (lambda_2 - lambda_1) of the minimum, so
    # the winner lies within a few covering radii of it
    assert np.median(ang) < cover
    assert ang.max() < 4 * cover, (ang.max(), cover)


def test_fibonacci_lattice_and_empty_pairs():
    c = gs.fibonacci_sphere(1000)
    np.testing.assert_allclose(np.linalg.norm(c, axis=1), 1.0, atol=1e-15)
    assert np.abs(c.mean(axis=0)).max() < 2e-3
    W = np.zeros((2, 9, 9))
    Rij = np.broadcast_to(np.eye(3), (2, 3, 3)).copy()
    prior = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    t, best, err = gs.grid_search(W, np.array([0, 0]), Rij, c, prior)
    np.testing.assert_array_equal(t, prior)
    np.testing.assert_array_equal(best, [-1, -1])
