"""Pins for the oracle's position, quantisation and keep rules.

The expected (cx, px) values below were worked out by hand from the rule
qx = floor(x*O + 1/2), cx = floor((qx + O/2)/O), px = qx - cx*O with x = u/du + nx/2; the
inputs are chosen so that every intermediate value is exact in binary floating point
(frequency = speed of light, so u equals the metre value; du = 1).
"""
import numpy as np
import pytest

from paper_0902_0915_amd.synth import C_LIGHT

NX = 64
F = np.array([C_LIGHT])  # u[lambda] == u[m]


def _one(orc, u, v=0.0, O=8, W=7, nx=NX, ny=NX, **kw):
    uvw = np.array([[u, v, 0.0]])
    pos, keep, counts = orc.positions(uvw, F, nx, ny, 1.0, 1.0, W, O, **kw)
    return pos[0], bool(keep[0]), counts


@pytest.mark.parametrize("u,cx,px", [
    (0.0, 32, 0),
    (0.0625, 32, 1),      # x*O + 1/2 = 257 exactly: the tie rounds up
    (-0.0625, 32, 0),     # 255.5 + 0.5 = 256
    (0.5, 33, -4),        # half a cell: next cell, phase -O/2
    (0.4375, 33, -4),     # 259.5 + 0.5 = 260
    (0.4374, 32, 3),
    (-3.3, 29, -2),       # 28.7 -> 229.6 + 0.5 -> 230 = 29*8 - 2
    (-0.5, 32, -4),       # 252 + 0.5 -> 252 = 32*8 - 4
    (10.9375, 43, 0),     # 42.9375*8 + 0.5 = 344 = 43*8
    (10.5, 43, -4),       # 42.5*8 + 0.5 -> 340 = 43*8 - 4
])
def test_quantisation_worked_examples(orc, u, cx, px):
    p, keep, _ = _one(orc, u)
    assert keep
    assert (p[0], p[2]) == (cx, px)
    assert (p[1], p[3]) == (32, 0)


def test_quantisation_v_axis_is_rows(orc):
    p, keep, _ = _one(orc, 0.0, v=-3.3)
    assert keep and tuple(p) == (32, 29, 0, -2)


@pytest.mark.parametrize("O", [1, 2, 3, 4, 8, 16])
def test_quantisation_error_bound(orc, O):
    rng = np.random.default_rng(O)
    u = rng.uniform(-20, 20, 2000)
    v = rng.uniform(-20, 20, 2000)
    uvw = np.stack([u, v, np.zeros_like(u)], axis=1)
    pos, keep, _ = orc.positions(uvw, F, NX, NX, 1.0, 1.0, 7, O)
    assert keep.all()
    lo, hi = -(O // 2), O - O // 2
    assert ((pos[:, 2] >= lo) & (pos[:, 2] < hi)).all()
    assert ((pos[:, 3] >= lo) & (pos[:, 3] < hi)).all()
    xq = pos[:, 0] + pos[:, 2] / O - NX / 2
    yq = pos[:, 1] + pos[:, 3] / O - NX / 2
    assert np.max(np.abs(xq - u)) <= 0.5 / O + 1e-12
    assert np.max(np.abs(yq - v)) <= 0.5 / O + 1e-12


def test_keep_rule_grid_edges(orc):
    # h = 3: a footprint must satisfy cx - 3 >= 0 and cx + 3 <= nx - 1.
    assert _one(orc, 3 - 32)[1]           # cx = 3
    assert not _one(orc, 2 - 32)[1]       # cx = 2
    assert _one(orc, 60 - 32)[1]          # cx = 60
    assert not _one(orc, 61 - 32)[1]      # cx = 61
    assert not _one(orc, 0.0, v=61 - 32)[1]
    p, keep, counts = _one(orc, 61 - 32)
    assert tuple(p) == (-1, -1, -1, -1) and counts == {"kept": 0, "flagged": 0, "outside": 1}
    # a wider kernel drops earlier
    assert not _one(orc, 60 - 32, W=9)[1]


def test_flags_weights_nonfinite(orc):
    uvw = np.array([[1.0, 1.0, 0.0], [2.0, 2.0, 0.0], [np.nan, 0.0, 0.0], [np.inf, 0.0, 0.0],
                    [3.0, 3.0, 0.0]])
    flags = np.array([0, 1, 0, 0, 0], dtype=np.uint8)
    weights = np.array([1.0, 1.0, 1.0, 1.0, 0.0])
    pos, keep, counts = orc.positions(uvw, F, NX, NX, 1.0, 1.0, 7, 8, flags=flags,
                                      weights=weights)
    assert keep.tolist() == [True, False, False, False, False]
    assert counts == {"kept": 1, "flagged": 2, "outside": 2}


def test_channel_scaling(orc):
    # u = u_m * f / c: doubling the frequency doubles the offset from the grid centre.
    uvw = np.array([[4.0, -2.0, 0.0]])
    freq = np.array([C_LIGHT, 2 * C_LIGHT])
    pos, keep, _ = orc.positions(uvw, freq, NX, NX, 1.0, 1.0, 7, 8)
    assert keep.all()
    assert tuple(pos[0]) == (36, 30, 0, 0) and tuple(pos[1]) == (40, 28, 0, 0)
