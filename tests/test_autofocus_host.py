"""Host-side pieces of the autofocus driver: spline basis, detrending, and the
L-BFGS ascent, checked on problems with known answers (no GPU)."""
import numpy as np
import pytest

from paper_2101_05888_amd.autofocus import _lbfgs_ascent, bspline_basis, detrended_rms, line_of_sight_frame


@pytest.mark.parametrize("n,spacing", [(256, 64), (256, 8), (100, 7.5), (17, 4)])
def test_bspline_partition_of_unity_and_reproduces_lines(n, spacing):
    B = bspline_basis(n, spacing)
    assert np.abs(B.sum(axis=1) - 1.0).max() < 1e-12
    # cubic B-splines reproduce polynomials up to degree 3
    t = np.arange(n, dtype=np.float64)
    for f in (t, (t - 20.0) ** 2 * 1e-3, (t - 5.0) ** 3 * 1e-5):
        w, *_ = np.linalg.lstsq(B, f, rcond=None)
        assert np.abs(B @ w - f).max() < 1e-9 * max(1.0, np.abs(f).max())


def test_detrended_rms_removes_line_exactly():
    n = 64
    t = np.arange(n, dtype=np.float64)
    wiggle = np.sin(0.7 * t)
    wiggle -= np.polyval(np.polyfit(t, wiggle, 1), t)
    err = np.stack([3.0 + 0.2 * t, -1.0 + 0.01 * t + wiggle], axis=1)
    r = detrended_rms(err)
    assert r[0] < 1e-12
    assert r[1] == pytest.approx(np.sqrt((wiggle ** 2).mean()), rel=1e-12)


def test_lbfgs_ascent_solves_ill_conditioned_quadratic():
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.normal(size=(12, 12)))
    A = Q @ np.diag(np.logspace(-3, 1, 12)) @ Q.T
    b = rng.normal(size=12)
    xs = np.linalg.solve(A, b)

    def vg(x, grad=True):
        return -0.5 * x @ A @ x + b @ x, (b - A @ x) if grad else None

    x = _lbfgs_ascent(vg, np.zeros(12), 400, 0.5, max_step=1e6)
    assert np.abs(x - xs).max() < 1e-5 * np.abs(xs).max()


def test_line_of_sight_frame_is_orthonormal_and_points_at_the_scene():
    tx = np.stack([np.arange(10) * 0.15, np.zeros(10), np.full(10, -10.0)], axis=1)
    R = line_of_sight_frame(tx, [0.7, 27.0, 0.0])
    assert np.allclose(R @ R.T, np.eye(3), atol=1e-15)
    assert R[1, 0] == 0.0 and R[1, 1] > 0 and R[1, 2] > 0     # z down: the scene is below the track
    assert R[1] @ np.array([0.0, 27.0, 10.0]) == pytest.approx(np.hypot(27.0, 10.0))
