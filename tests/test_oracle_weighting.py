"""Pins of the oracle's density weighting (uniform and Briggs robust; outside the paper, an
imaging variant of its gridding step): a hand-worked case, the unit sum of uniform weights in
every occupied cell, and the published limits of robust weighting (natural as R -> +inf,
uniform as R -> -inf, each up to a constant factor)."""
import numpy as np


def _pos(cells):
    pos = np.array([[x, y, 0, 0] for x, y in cells], dtype=np.int32)
    return pos, np.ones(len(cells), dtype=bool)


def test_hand_worked_uniform_and_robust(orc):
    # three samples in cell A = (2, 3) with weights 1, 1, 2; one in cell B = (5, 1) with weight 1
    pos, keep = _pos([(2, 3), (2, 3), (5, 1), (2, 3)])
    w = np.array([1.0, 1.0, 1.0, 2.0])
    u = orc.density_weights(pos, keep, 8, 8, w, "uniform")
    np.testing.assert_allclose(u, [0.25, 0.25, 1.0, 0.5], atol=1e-15)
    # robust R = 0: f^2 = 25 / ((4^2 + 1^2) / 5) = 125 / 17
    r = orc.density_weights(pos, keep, 8, 8, w, "robust", 0.0)
    f2 = 125.0 / 17.0
    np.testing.assert_allclose(r, [1 / (1 + 4 * f2), 1 / (1 + 4 * f2), 1 / (1 + f2), 2 / (1 + 4 * f2)],
                               rtol=1e-14)


def test_uniform_weights_sum_to_one_per_cell_and_dropped_are_zero(orc):
    rng = np.random.default_rng(1)
    n = 3000
    pos = np.stack([rng.integers(0, 16, n), rng.integers(0, 12, n), np.zeros(n, int), np.zeros(n, int)], axis=1)
    keep = rng.random(n) > 0.1
    w = rng.uniform(0.1, 3.0, n)
    u = orc.density_weights(pos, keep, 16, 12, w, "uniform")
    assert np.all(u[~keep] == 0)
    cell = pos[:, 1] * 16 + pos[:, 0]
    sums = np.bincount(cell[keep], weights=u[keep], minlength=16 * 12)
    occupied = np.bincount(cell[keep], minlength=16 * 12) > 0
    np.testing.assert_allclose(sums[occupied], 1.0, rtol=1e-12)


def test_robust_limits(orc):
    rng = np.random.default_rng(2)
    n = 2000
    pos = np.stack([rng.integers(0, 10, n), rng.integers(0, 10, n), np.zeros(n, int), np.zeros(n, int)], axis=1)
    keep = np.ones(n, dtype=bool)
    w = rng.uniform(0.5, 1.5, n)
    nat = orc.density_weights(pos, keep, 10, 10, w, "robust", 8.0)
    np.testing.assert_allclose(nat / nat.mean(), w / w.mean(), rtol=1e-10)
    uni = orc.density_weights(pos, keep, 10, 10, w, "robust", -8.0)
    ref = orc.density_weights(pos, keep, 10, 10, w, "uniform")
    np.testing.assert_allclose(uni / uni.mean(), ref / ref.mean(), rtol=1e-8)
