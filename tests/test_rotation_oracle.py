"""Pins of the FP64 rotation-averaging oracle against what the paper and the
mathematics fix (Sec. 3.3 "Global Rotation", eq. rotation-objective and the
geodesic distance; appendix on rotation initialisation), independent of the
oracle's own formulas."""
import numpy as np
import pytest

from oracle import rotation as ra
from paper_2505_04612_amd import synth


def _rz(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _rx(a):
    c, s = np.cos(a), np.sin(a)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


def _params(R):
    return np.concatenate([R[:, :, 0], R[:, :, 1]], axis=1)


@pytest.fixture(scope="module")
def tiny():
    return synth.tiny()


def test_hand_values_geodesic():
    # a rotation by angle a about any axis is at geodesic distance a from I
    for a in (0.0, 0.3, 1.2, 3.0):
        assert ra.geodesic(_rz(a), np.eye(3)) == pytest.approx(a, abs=1e-7 if a == 0 else 1e-12)
        assert ra.geodesic(_rx(a) @ _rz(0.4), _rz(0.4)) == pytest.approx(a, abs=1e-7 if a == 0 else 1e-12)
    # two cameras: R_0 = I, R_1 = Rz(0.7), measured relative rotation I
    R = np.stack([np.eye(3), _rz(0.7)])
    assert ra.loss(_params(R), np.array([[0, 1]]), np.eye(3)[None]) == pytest.approx(0.7, abs=1e-12)


def test_zero_at_truth_and_global_rotation_invariance(tiny):
    inp = synth.rotation_inputs(tiny, sigma_deg=0.0, outlier_frac=0.0)
    th = _params(tiny.R_gt)
    assert ra.loss(th, tiny.pairs, inp.R_rel) < 1e-7          # arccos near 1 resolves ~1e-8 rad
    noisy = synth.rotation_inputs(tiny)
    L = ra.loss(th, tiny.pairs, noisy.R_rel)
    G = _rx(0.9) @ _rz(-2.0)
    assert ra.loss(_params(tiny.R_gt @ G), tiny.pairs, noisy.R_rel) == pytest.approx(L, rel=1e-12)


def test_gradient_central_differences(tiny):
    inp = synth.rotation_inputs(tiny)
    rng = np.random.default_rng(3)
    th = _params(tiny.R_gt) + 0.05 * rng.normal(size=(tiny.R_gt.shape[0], 6))
    L, g = ra.loss_grad(th, tiny.pairs, inp.R_rel)
    assert L == pytest.approx(ra.loss(th, tiny.pairs, inp.R_rel), rel=1e-14)
    h = 1e-7
    for _ in range(10):
        d = rng.normal(size=th.shape)
        fd = (ra.loss(th + h * d, tiny.pairs, inp.R_rel) - ra.loss(th - h * d, tiny.pairs, inp.R_rel)) / (2 * h)
        an = (g * d).sum()
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (fd, an)


def test_column_system_is_the_sum_of_squares(tiny):
    inp = synth.rotation_inputs(tiny)
    N = tiny.R_gt.shape[0]
    A = ra.column_system(tiny.pairs, inp.R_rel, N)
    rng = np.random.default_rng(4)
    x = rng.normal(size=(N, 3))
    direct = sum(float(np.sum((x[j] - Q @ x[i]) ** 2)) for (i, j), Q in zip(tiny.pairs, inp.R_rel))
    assert float(x.ravel() @ A @ x.ravel()) == pytest.approx(direct, rel=1e-12)
    np.testing.assert_allclose(A, A.T, atol=1e-14)


def test_noise_free_initialisation_is_exact_up_to_a_global_rotation(tiny):
    inp = synth.rotation_inputs(tiny, sigma_deg=0.0, outlier_frac=0.0)
    N = tiny.R_gt.shape[0]
    R, info = ra.initialise(tiny.pairs, inp.R_rel, N)
    w = np.linalg.eigvalsh(info["A"])
    # the first columns of any rotated truth solve the problem exactly: a
    # three-dimensional null space, then a gap
    assert np.abs(w[:3]).max() < 1e-10 and w[3] > 0.1
    # the solution is R_i v for one unit v: the first columns are the truth
    # applied to the same vector in every camera
    c1 = R[:, :, 0]
    v = tiny.R_gt[0].T @ c1[0]
    np.testing.assert_allclose(np.einsum("nab,b->na", tiny.R_gt, v), c1, atol=1e-9)
    # proper rotations, related to the truth by one global rotation
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)
    # (arccos of 1 - 4e-16 is already 1.6e-6 deg: the angle metric resolves
    # no finer; the matrix comparison below is the strict one)
    assert ra.relative_rotation_errors(R, tiny.R_gt, tiny.pairs).max() < 1e-5
    G = tiny.R_gt[0].T @ R[0]
    np.testing.assert_allclose(tiny.R_gt @ G, R, atol=1e-9)


def test_second_column_penalty_and_orthogonality(tiny):
    inp = synth.rotation_inputs(tiny)
    N = tiny.R_gt.shape[0]
    R, info = ra.initialise(tiny.pairs, inp.R_rel, N)
    # the penalised problem's matrix: pair term / |P| plus (1/N) c1 c1^T blocks
    c1 = R[:, :, 0]
    rng = np.random.default_rng(8)
    y = rng.normal(size=(N, 3))
    direct = (sum(float(np.sum((y[j] - Q @ y[i]) ** 2)) for (i, j), Q in zip(tiny.pairs, inp.R_rel))
              / len(tiny.pairs) + float(np.sum(np.sum(c1 * y, axis=1) ** 2)) / N)
    assert float(y.ravel() @ info["B"] @ y.ravel()) == pytest.approx(direct, rel=1e-12)
    np.testing.assert_allclose(np.einsum("nab,nac->nbc", R, R), np.broadcast_to(np.eye(3), (N, 3, 3)), atol=1e-12)


def test_solve_recovers_truth_from_a_perturbed_start(tiny):
    inp = synth.rotation_inputs(tiny, sigma_deg=0.0, outlier_frac=0.0)
    rng = np.random.default_rng(9)
    R0 = np.stack([_rx(a) @ _rz(b) @ R for a, b, R in zip(rng.uniform(-0.08, 0.08, 20), rng.uniform(-0.08, 0.08, 20),
                                                           tiny.R_gt)])
    th, trace = ra.solve(_params(R0), tiny.pairs, inp.R_rel, 500, 1e-2)
    assert trace[-1] < 0.02 * trace[0]
    assert ra.relative_rotation_errors(ra.rotations(th), tiny.R_gt, tiny.pairs).max() < 0.01


def test_relative_rotation_errors_metric():
    R = np.stack([np.eye(3), _rz(0.5), _rx(1.0)])
    pairs = np.array([[0, 1], [1, 2]])
    assert ra.relative_rotation_errors(R, R @ _rx(0.3), pairs).max() < 1e-6
    R2 = R.copy()
    R2[1] = _rz(0.2) @ R[1]
    e = ra.relative_rotation_errors(R, R2, pairs)
    assert e[0] == pytest.approx(np.degrees(0.2), abs=1e-9)
