"""Pins for the oracle's pointwise forms (grid_cells, degrid_groups), used where a grid is too
large for the whole-grid oracle: they must agree with the pinned scatter and gather loops
(oracle.c, a separate implementation) at every sampled output, with and without weights."""
import numpy as np
import pytest

import oracle as orc
from paper_0902_0915_amd import synth


@pytest.fixture(scope="module")
def case():
    wl = synth.mwa_scale(seed=2011, nant=24, nchan=4, ntime=2, npol=4, n=128, nsrc=5)
    rng = np.random.default_rng(3)
    w = rng.uniform(0.5, 1.5, wl.ngroups)
    pos, keep, _ = orc.positions(wl.uvw, wl.freq, wl.nx, wl.ny, wl.du, wl.dv, wl.W, wl.O)
    return wl, w, pos, keep, rng


@pytest.mark.parametrize("weighted", [False, True])
def test_grid_cells_match_whole_grid(case, weighted):
    wl, w, pos, keep, rng = case
    weights = w if weighted else None
    G = orc.grid(pos, keep, wl.vis, wl.nx, wl.ny, wl.W, wl.O, nchan=wl.nchan, weights=weights)
    # every cell of a band through the centre, plus random cells anywhere (empty ones too)
    band = [(x, y) for y in range(60, 68) for x in range(wl.nx)]
    rnd = [tuple(c) for c in rng.integers(0, [wl.nx, wl.ny], size=(300, 2))]
    cells = np.array(band + rnd)
    got = orc.grid_cells(pos, keep, wl.vis, cells, wl.nx, wl.W, wl.O, weights=weights)
    ref = G[:, cells[:, 1], cells[:, 0]]
    assert np.abs(ref).max() > 0
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("weighted", [False, True])
def test_degrid_groups_match_whole_adjoint(case, weighted):
    wl, w, pos, keep, rng = case
    weights = w if weighted else None
    G = rng.standard_normal((4, wl.ny, wl.nx)) + 1j * rng.standard_normal((4, wl.ny, wl.nx))
    ref = orc.degrid(pos, keep, G, wl.W, wl.O, nchan=wl.nchan, weights=weights)
    kept = np.flatnonzero(keep)
    sel = rng.choice(kept, size=min(500, len(kept)), replace=False)
    got = orc.degrid_groups(pos, G, sel, wl.W, wl.O, weights=weights)
    assert np.allclose(got, ref[sel], rtol=1e-12, atol=1e-12 * np.abs(ref).max())
