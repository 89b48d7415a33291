"""Pins of the FP64 translation-averaging oracle against what the paper and the
mathematics fix (Sec. 3.3 "Global Translation", eq. global-translation-objective;
App. "Multiple Initializations"), independent of the oracle's own formulas."""
import numpy as np
import pytest

from oracle import translation as ta
from paper_2505_04612_amd import synth


def _centres(sc):
    return -np.einsum("nba,nb->na", sc.R_gt, sc.t_gt)


@pytest.fixture(scope="module")
def tiny():
    return synth.tiny()


def test_target_is_the_unit_vector_from_centre_i_to_centre_j(tiny):
    # the paper names o^{i->j} the normalised vector from camera i's centre to
    # camera j's, in world coordinates: with exact relative translations the
    # printed formula -R_j^T t^{i->j} must give exactly that
    inp = synth.translation_inputs(tiny, sigma_deg=0.0, outlier_frac=0.0)
    d = ta.target_directions(tiny.R_gt, inp.t_rel, tiny.pairs)
    o = _centres(tiny)
    want = o[tiny.pairs[:, 1]] - o[tiny.pairs[:, 0]]
    want /= np.linalg.norm(want, axis=1, keepdims=True)
    np.testing.assert_allclose(d, want, atol=1e-12)


def test_hand_value_two_cameras():
    # o_0 = 0, o_1 = (2,0,0): unit direction (1,0,0); target (0,1,0):
    # L1 distance |1-0| + |0-1| + 0 = 2 over one pair.  dL/du = (1,-1,0);
    # projected off u: (0,-1,0); divided by |s| = 2: camera 1 gets (0,-0.5,0)
    # and camera 0 the opposite.
    o = np.array([[0.0, 0.0, 0.0], [2.0, 0.0, 0.0]])
    pairs = np.array([[0, 1]])
    d = np.array([[0.0, 1.0, 0.0]])
    L, g = ta.loss_grad(o, pairs, d)
    assert L == 2.0
    np.testing.assert_array_equal(g, [[0.0, 0.5, 0.0], [0.0, -0.5, 0.0]])


def test_zero_at_truth_and_similarity_invariance(tiny):
    inp = synth.translation_inputs(tiny, sigma_deg=0.0, outlier_frac=0.0)
    d = ta.target_directions(tiny.R_gt, inp.t_rel, tiny.pairs)
    o = _centres(tiny)
    assert ta.loss(o, tiny.pairs, d) < 1e-14
    rng = np.random.default_rng(5)
    o2 = rng.normal(size=o.shape)
    L = ta.loss(o2, tiny.pairs, d)
    for a, c in [(0.3, np.array([1.0, -2.0, 0.5])), (7.0, np.zeros(3))]:
        assert abs(ta.loss(a * o2 + c, tiny.pairs, d) - L) < 1e-12 * L
    # a reflection flips every direction: the truth becomes the worst case
    assert ta.loss(-o, tiny.pairs, d) > 1.0


def test_gradient_invariants_and_central_differences(tiny):
    inp = synth.translation_inputs(tiny)
    d = ta.target_directions(tiny.R_gt, inp.t_rel, tiny.pairs)
    o = inp.init[0]
    L, g = ta.loss_grad(o, tiny.pairs, d)
    # translation invariance: the gradients sum to 0; scale invariance:
    # sum_i o_i . g_i = 0
    assert np.abs(g.sum(axis=0)).max() < 1e-14
    assert abs((o * g).sum()) < 1e-14
    # central differences along random directions (the test point is away
    # from the L1 kinks by far more than the step)
    u = ta.pair_terms(o, tiny.pairs, d)[2]
    assert np.abs(u - d).min() > 1e-5
    rng = np.random.default_rng(6)
    h = 1e-8
    for _ in range(10):
        dirn = rng.normal(size=o.shape)
        fd = (ta.loss(o + h * dirn, tiny.pairs, d) - ta.loss(o - h * dirn, tiny.pairs, d)) / (2 * h)
        an = (g * dirn).sum()
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_coincident_centres_add_nothing():
    o = np.array([[1.0, 2.0, 3.0], [1.0, 2.0, 3.0], [0.0, 0.0, 0.0]])
    pairs = np.array([[0, 1], [0, 2]])
    d = np.array([[1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    L, g = ta.loss_grad(o, pairs, d)
    u = -o[0] / np.linalg.norm(o[0])
    assert L == pytest.approx(np.abs(u - d[1]).sum() / 2, abs=1e-15)
    # the coincident pair leaves camera 1 without gradient
    assert np.all(g[1] == 0.0)


def test_noise_free_solve_recovers_the_centres_from_random_starts(tiny):
    inp = synth.translation_inputs(tiny, sigma_deg=0.0, outlier_frac=0.0, runs=2)
    d = ta.target_directions(tiny.R_gt, inp.t_rel, tiny.pairs)
    gt = ta.normalize(_centres(tiny))
    for r in range(2):
        o, trace = ta.solve(inp.init[r], tiny.pairs, d, 1000, 3e-2)
        assert trace[-1] < 1e-2 * trace[0]
        assert np.linalg.norm(ta.normalize(o) - gt, axis=1).max() < 2e-3


def test_normalize_closed_form():
    rng = np.random.default_rng(7)
    o = rng.normal(size=(50, 3)) * 4.0 + 3.0
    n = ta.normalize(o)
    assert np.abs(n.mean(axis=0)).max() < 1e-14
    assert abs(np.linalg.norm(n, axis=1).mean() - 1.0) < 1e-14
    # a similarity of the input changes nothing
    np.testing.assert_allclose(ta.normalize(0.01 * o - 5.0), n, atol=1e-13)
    # all centres equal: centred only
    np.testing.assert_array_equal(ta.normalize(np.ones((4, 3))), np.zeros((4, 3)))


def test_merge_aligns_similar_runs_and_replaces_a_displaced_camera(tiny):
    inp = synth.translation_inputs(tiny, sigma_deg=0.0, outlier_frac=0.0)
    d = ta.target_directions(tiny.R_gt, inp.t_rel, tiny.pairs)
    o = _centres(tiny)
    runs = np.stack([2.0 * o + 1.0, 0.5 * o - 3.0, 10.0 * o])
    merged, choice, cam = ta.merge(runs, tiny.pairs, d)
    np.testing.assert_allclose(merged, ta.normalize(o), atol=1e-12)
    assert cam.max() < 1e-12
    # identical runs score identically: the lowest run index is taken
    merged, choice, cam = ta.merge(np.stack([o, o, o]), tiny.pairs, d)
    np.testing.assert_array_equal(choice, 0)
    # displace camera 3 in run 0: its own score rises, so it is taken from
    # another run, and lands where the truth says
    bad = runs.copy()
    bad[0, 3] += np.array([5.0, -5.0, 5.0])
    merged, choice, cam = ta.merge(bad, tiny.pairs, d)
    assert choice[3] != 0
    assert cam[0, 3] > 0.1 and cam[choice[3], 3] < 1e-12
    np.testing.assert_allclose(merged[3], ta.normalize(o)[3], atol=1e-12)


def test_camera_without_pairs_takes_the_first_run():
    pairs = np.array([[0, 1]])
    d = np.array([[1.0, 0.0, 0.0]])
    runs = np.array([[[0.0, 0, 0], [1.0, 0, 0], [9.0, 9, 9]],
                     [[0.0, 0, 0], [0.0, 1, 0], [1.0, 1, 1]]])
    merged, choice, cam = ta.merge(runs, pairs, d)
    assert list(choice) == [0, 0, 0]
    assert np.all(cam[:, 2] == 0.0)
