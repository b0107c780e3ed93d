"""The plan's gridding order (the sort by uv tile standing for the memory structures that
Section 3.2 says the port needed), read back through mw_plan_order and checked against the
plan's own positions: a permutation of the kept groups, tile-major, each cell's groups
together, row sub-positions ascending within a cell, and equal keys in input order (the sort
is stable). With more groups than grid cells the radial cell ranks come from the per-cell
table, otherwise from the per-group evaluation; both must give these properties."""
import numpy as np
import pytest

from paper_0902_0915_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mw():
    import torch
    assert torch.cuda.is_available()
    from paper_0902_0915_amd import mwagrid
    return mwagrid


def _order(mw, wl, **tuning):
    spec = mw.InstanceSpec.from_workload(wl, with_ants=False)
    with mw.Plan(spec, tuning=tuning) as plan:
        info = plan.info(0)
        return plan.order(0), plan.positions(0), info


def _check_order(wl, perm, pos, info, order, tile):
    keep = pos[:, 0] >= 0
    assert info["nkept"] == int(keep.sum()) == perm.size
    np.testing.assert_array_equal(np.sort(perm), np.flatnonzero(keep))  # a permutation of the kept
    cx, cy, py = pos[perm, 0], pos[perm, 1], pos[perm, 3]
    ntx = (wl.nx + tile - 1) // tile
    t = (cy // tile) * ntx + cx // tile
    assert np.all(np.diff(t) >= 0)  # tile-major
    same_tile = t[1:] == t[:-1]
    if order == 2:
        assert np.all(perm[1:][same_tile] > perm[:-1][same_tile])  # input order within a tile
        return
    cell = cy * wl.nx + cx
    start = np.r_[True, cell[1:] != cell[:-1]]
    assert np.unique(cell[start]).size == int(start.sum())  # each cell's groups together
    same_cell = ~start[1:]
    assert np.all(py[1:][same_cell] >= py[:-1][same_cell])  # row sub-positions ascending
    same_key = same_cell & (py[1:] == py[:-1])
    assert np.all(perm[1:][same_key] > perm[:-1][same_key])  # stable: equal keys in input order
    if order == 1:  # cells row by row within a tile
        lr = (cy % tile) * tile + cx % tile
        assert np.all(lr[1:][same_tile] >= lr[:-1][same_tile])


@pytest.mark.parametrize("n,order,tile", [(512, 3, 8), (128, 3, 8), (128, 3, 16), (256, 1, 8), (256, 2, 8)])
def test_gridding_order(mw, n, order, tile):
    rng = np.random.default_rng(90 + n + order)
    wl = synth.mwa_scale(seed=2090, nant=48, nchan=8, ntime=2, npol=1, n=n, nsrc=5, make_vis=False)
    wl.flags = (rng.random(wl.ngroups) < 0.1).astype(np.uint8)
    if order == 3 and n == 128:
        assert wl.ngroups > n * n  # more groups than cells: the rank table
    perm, pos, info = _order(mw, wl, variant=4, tile=tile, order=order)
    assert info["tile"] == tile and info["order"] == order
    _check_order(wl, perm, pos, info, order, tile)


def test_gridding_order_of_a_batched_plan(mw):
    """A plan of four instances sorts each on a worker thread, once the batch has chosen its
    tile: every instance's order has the same properties at that tile."""
    jobs = [synth.mwa_scale(seed=2091 + k, nant=24 + 8 * k, nchan=4 + 2 * k, ntime=2, npol=1, n=n,
                            nsrc=3, make_vis=False) for k, n in enumerate((256, 512, 128, 256))]
    specs = [mw.InstanceSpec.from_workload(j, with_ants=False) for j in jobs]
    with mw.Plan(specs) as plan:
        for k, wl in enumerate(jobs):
            info = plan.info(k)
            _check_order(wl, plan.order(k), plan.positions(k), info, info["order"], info["tile"])

