"""Pins of the oracle's calibration steps (Section 2: per-antenna complex gains from a linear
least-squares fit to catalogue sources; Section 2.1: catalogue sources measured and removed
in decreasing order of predicted flux, each measurement constraining the gains; Table 1,
"CML"). Nothing here re-types the oracle's sums: prediction is pinned by closed forms, its
symmetry and the position of its image peak (through the pinned gridder and transform); the
gain solver by exact recovery of known gains from noise-free data, its fixed point and the
meaning of a zero weight; the peeling loop by exact removal of a single source and its
independence of the catalogue's order."""
import numpy as np
import pytest

C = 299_792_458.0


def _array(rng, nant=12, ntime=3):
    pos = rng.uniform(-400.0, 400.0, (nant, 3))
    pos[:, 2] *= 0.02
    a1, a2 = np.triu_indices(nant, 1)
    rows = []
    for t in range(ntime):
        rot = 0.05 * t
        R = np.array([[np.cos(rot), -np.sin(rot), 0], [np.sin(rot), np.cos(rot), 0], [0, 0, 1.0]])
        rows.append((pos[a1] - pos[a2]) @ R.T)
    uvw = np.concatenate(rows)
    return uvw, np.tile(a1, ntime), np.tile(a2, ntime), nant


def test_predict_source_at_phase_centre_is_its_flux(orc):
    rng = np.random.default_rng(1)
    uvw = rng.uniform(-500, 500, (40, 3))
    V = orc.predict(uvw, np.array([150e6, 160e6]), [[0.0, 0.0, 2.5]], npol=4)
    assert V.shape == (80, 4)
    np.testing.assert_allclose(V[:, [0, 3]], 2.5, atol=1e-15)
    np.testing.assert_array_equal(V[:, [1, 2]], 0)


def test_predict_whole_turns_and_hermitian_symmetry(orc):
    # u = 100 wavelengths, l = 0.01: one whole turn of phase, so V = S; half a turn at l = 0.005
    f = 150e6
    uvw = np.array([[100.0 * C / f, 0.0, 0.0]])
    np.testing.assert_allclose(orc.predict(uvw, [f], [[0.01, 0.0, 3.0]])[0, 0], 3.0, atol=1e-12)
    np.testing.assert_allclose(orc.predict(uvw, [f], [[0.005, 0.0, 3.0]])[0, 0], -3.0, atol=1e-12)
    rng = np.random.default_rng(2)
    uvw = rng.uniform(-800, 800, (30, 3))
    src = [[0.05, -0.02, 1.0], [-0.1, 0.07, 0.4]]
    a = orc.predict(uvw, [140e6, 170e6], src)
    b = orc.predict(-uvw, [140e6, 170e6], src)
    np.testing.assert_allclose(b, np.conj(a), atol=1e-12)


def test_predicted_source_images_at_its_pixel(orc):
    # the dirty image of one predicted source (w = 0) peaks at x = n/2 + l n du, y = n/2 + m n dv
    rng = np.random.default_rng(3)
    n, du = 128, 4.0
    f = 150e6
    uv = rng.uniform(-0.35 * n * du, 0.35 * n * du, (3000, 2))
    uvw = np.concatenate([uv, np.zeros((3000, 1))], axis=1) * (C / f)
    px, py = 75, 50
    l, m = (px - n / 2) / (n * du), (py - n / 2) / (n * du)
    V = orc.predict(uvw, [f], [[l, m, 1.0]])
    pos, keep, _ = orc.positions(uvw, np.array([f]), n, n, du, du, 7, 8)
    img = orc.image(orc.grid(pos, keep, V, n, n, 7, 8), W=7, correct=True)
    y, x = np.unravel_index(np.argmax(np.abs(img[0])), img[0].shape)
    assert (x, y) == (px, py)
    assert abs(img[0, py, px] - keep.sum()) < 0.02 * keep.sum()


def test_stefcal_recovers_known_gains_from_noise_free_data(orc):
    rng = np.random.default_rng(4)
    uvw, a1, a2, nant = _array(rng)
    freq = np.array([150e6, 155e6])
    M = orc.predict(uvw, freq, [[0.02, 0.01, 3.0], [-0.05, 0.03, 1.0]], npol=2)
    g_true = (1 + 0.2 * rng.standard_normal(nant)) * np.exp(1j * rng.uniform(-1, 1, nant))
    rows = np.arange(M.shape[0]) // 2
    V = (g_true[a1[rows]] * np.conj(g_true[a2[rows]]))[:, None] * M
    g, rel = orc.stefcal(V, M, a1, a2, nant, 2, niter=80)
    g = g * np.exp(-1j * np.angle(g[0] / g_true[0]))  # the common phase is not determined
    np.testing.assert_allclose(g, g_true, rtol=0, atol=1e-9)
    assert rel < 1e-9
    # the true gains are a fixed point of one iteration
    g1, _ = orc.stefcal(V, M, a1, a2, nant, 2, g0=g_true, niter=1)
    np.testing.assert_allclose(g1, g_true, atol=1e-13)


def test_stefcal_zero_weight_excludes_a_sample(orc):
    rng = np.random.default_rng(5)
    uvw, a1, a2, nant = _array(rng, nant=8, ntime=2)
    M = orc.predict(uvw, [150e6], [[0.03, -0.02, 2.0]])
    V = M * (1.0 + 0.3 * (rng.standard_normal(M.shape) + 1j * rng.standard_normal(M.shape)))
    w = (rng.random(M.shape[0]) > 0.3).astype(np.float64)
    keep = w > 0
    ga, _ = orc.stefcal(V, M, a1, a2, nant, 1, niter=7, weights=w)
    gb, _ = orc.stefcal(V[keep], M[keep], a1[keep], a2[keep], nant, 1, niter=7)
    np.testing.assert_allclose(ga, gb, atol=1e-13)
    # corrupting the excluded samples changes nothing
    V2 = V.copy()
    V2[~keep] = 1e6
    gc, _ = orc.stefcal(V2, M, a1, a2, nant, 1, niter=7, weights=w)
    np.testing.assert_allclose(gc, ga, atol=1e-13)


def test_peel_removes_a_single_source_exactly(orc):
    rng = np.random.default_rng(6)
    uvw, a1, a2, nant = _array(rng)
    freq = np.array([150e6, 152e6, 154e6])
    src = np.array([[0.04, -0.03, 5.0]])
    M = orc.predict(uvw, freq, src, npol=4)
    g_true = (1 + 0.1 * rng.standard_normal(nant)) * np.exp(1j * rng.uniform(-0.5, 0.5, nant))
    rows = np.arange(M.shape[0]) // 3
    V = (g_true[a1[rows]] * np.conj(g_true[a2[rows]]))[:, None] * M
    R, G, rel, order = orc.peel(V, uvw, freq, a1, a2, nant, src, npol=4, niter=80)
    assert np.linalg.norm(R) < 1e-9 * np.linalg.norm(V)
    g = G[0] * np.exp(-1j * np.angle(G[0, 0] / g_true[0]))
    np.testing.assert_allclose(g, g_true, atol=1e-9)


def test_peel_order_is_by_decreasing_flux_whatever_the_catalogue_order(orc):
    rng = np.random.default_rng(7)
    uvw, a1, a2, nant = _array(rng, nant=10)
    freq = np.array([150e6, 151e6])
    src = np.array([[0.04, -0.03, 1.0], [-0.02, 0.05, 8.0], [0.01, 0.02, -3.0]])
    V = orc.predict(uvw, freq, src) + 0.05 * (rng.standard_normal((uvw.shape[0] * 2, 1)) + 0j)
    R1, G1, r1, o1 = orc.peel(V, uvw, freq, a1, a2, nant, src, niter=6)
    assert o1 == [1, 2, 0]
    perm = [2, 0, 1]
    R2, G2, r2, o2 = orc.peel(V, uvw, freq, a1, a2, nant, src[perm], niter=6)
    np.testing.assert_allclose(R2, R1, atol=1e-12)
    np.testing.assert_allclose(G2, G1[perm], atol=1e-12)
    # a source of zero flux is measured as nothing and removes nothing
    R3, G3, _, _ = orc.peel(V, uvw, freq, a1, a2, nant, np.vstack([src, [[0.1, 0.1, 0.0]]]), niter=6)
    np.testing.assert_allclose(R3, R1, atol=1e-12)
    np.testing.assert_array_equal(G3[3], 1.0)
