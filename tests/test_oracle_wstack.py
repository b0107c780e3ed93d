"""Pins of the oracle's w-stacking (an imaging variant outside the paper): the stacked image
approaches the brute-force direct transform that includes the w-term, more closely with more
planes (a wrong sign of the plane phase makes it worse instead), the planes partition the kept
groups, and a plane at w = 0 adds its image unchanged."""
import numpy as np

C = 299_792_458.0


def _noncoplanar(rng, n=300):
    # a phase centre far from the zenith: w grows with u and v (metres = wavelengths at f = c)
    uv = rng.uniform(-24.0, 24.0, (n, 2))
    w = 0.9 * uv[:, 0] + 0.4 * uv[:, 1] + rng.uniform(-3, 3, n)
    return np.concatenate([uv, w[:, None]], axis=1)


def _stacked(orc, uvw, V, nw, n, du, edges):
    f = np.array([C])
    imgs, wp = [], []
    for k in range(nw):
        lo, hi = edges[k], edges[k + 1]
        pos, keep, _ = orc.positions(uvw, f, n, n, du, du, 7, 8, wrange=(lo, hi))
        G = orc.grid(pos, keep, V, n, n, 7, 8)
        imgs.append(orc.image(G, W=7, correct=True))
        wp.append(0.5 * (lo + hi))
    return orc.wstack_combine(np.array(imgs), np.array(wp), du, du)


def test_stacked_image_converges_to_the_direct_transform_with_w(orc):
    rng = np.random.default_rng(1)
    uvw = _noncoplanar(rng)
    n, du = 64, 1.0
    src = [[0.12, -0.08, 1.0], [-0.15, 0.1, 0.7], [0.05, 0.16, 0.5]]
    V = orc.predict(uvw, [C], src)
    wmin, wmax = uvw[:, 2].min(), uvw[:, 2].max() + 1e-9
    # direct transform including the w-term on the inner half of the field
    q = np.arange(n // 4, 3 * n // 4)
    l = (q - n // 2) / (n * du)
    L, M = np.meshgrid(l, l)
    N1 = np.sqrt(1 - L ** 2 - M ** 2) - 1
    D = np.zeros_like(L, dtype=np.complex128)
    for (u, v, w), val in zip(uvw, V[:, 0]):
        D += val * np.exp(2j * np.pi * (u * L + v * M + w * N1))
    errs = []
    for nw in (1, 4, 16, 64):
        edges = np.linspace(wmin, wmax, nw + 1)
        I = _stacked(orc, uvw, V, nw, n, du, edges)[0][np.ix_(q, q)]
        errs.append(np.linalg.norm(I - D) / np.linalg.norm(D))
    assert errs[0] > 0.3
    assert errs[0] > errs[1] > errs[2] > errs[3], errs
    assert errs[3] < 0.06, errs  # the floor is the O = 8 position quantisation


def test_planes_partition_the_kept_groups(orc):
    rng = np.random.default_rng(2)
    uvw = _noncoplanar(rng, 500)
    f = np.array([C, 1.1 * C])
    _, keep_all, _ = orc.positions(uvw, f, 64, 64, 1.0, 1.0, 7, 8)
    wl = (uvw[:, 2:3] * f[None, :]).reshape(-1) / C
    edges = np.linspace(wl.min(), wl.max() + 1e-9, 7)
    total = np.zeros(keep_all.shape, dtype=int)
    for k in range(6):
        _, keep, counts = orc.positions(uvw, f, 64, 64, 1.0, 1.0, 7, 8, wrange=(edges[k], edges[k + 1]))
        total += keep
        assert counts["flagged"] == np.sum((wl < edges[k]) | (wl >= edges[k + 1]))
    np.testing.assert_array_equal(total, keep_all.astype(int))


def test_plane_at_w_zero_is_added_unchanged(orc):
    rng = np.random.default_rng(3)
    z = rng.standard_normal((2, 1, 8, 8)) + 1j * rng.standard_normal((2, 1, 8, 8))
    out = orc.wstack_combine(z, np.array([0.0, 0.0]), 0.5, 0.5)
    np.testing.assert_allclose(out, z[0] + z[1], atol=1e-15)
