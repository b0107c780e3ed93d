"""Parity at the MWA-scale size and in the launch configuration bench.py times (512 antennas,
133,955,584 visibilities, 2048^2 x 4 grid, W = 7, O = 8, default launch). The whole grid is
too large for the oracle's scatter loop in a test, so sampled cells and sampled visibilities
are computed one by one (oracle.grid_cells, oracle.degrid_groups); the image of the GPU grid
is checked whole against the oracle's FFT."""
import numpy as np
import pytest

import oracle as orc
from paper_0902_0915_amd import synth
from _util import nl2, to_host

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def full():
    import torch
    assert torch.cuda.is_available()
    from paper_0902_0915_amd import mwagrid
    wl = synth.mwa_scale(device="cuda")
    spec = mwagrid.InstanceSpec.from_workload(wl, with_ants=False)
    with mwagrid.Plan(spec) as plan:
        info = plan.info(0)
        G = plan.grid(wl.vis)
        img = plan.image(G, direction=1, correct=False)
        back = plan.degrid(G)
        torch.cuda.synchronize()
        out = dict(info=info, G=to_host(G), img=to_host(img), back=to_host(back))
    out["vis"] = wl.vis.cpu().numpy()
    out["wl"] = wl
    pos, keep, counts = orc.positions(wl.uvw, wl.freq, wl.nx, wl.ny, wl.du, wl.dv, wl.W, wl.O)
    out.update(pos=pos, keep=keep, counts=counts)
    return out


def test_full_size_launch_is_the_benchmarked_one(full):
    info = full["info"]
    assert info["ngroups"] == 33_488_896 and full["vis"].shape == (33_488_896, 4)
    assert info["variant"] == 4 and info["flush"] == 2 and info["tile"] == 8
    assert info["nkept"] == int(full["keep"].sum())


def test_full_size_grid_sampled_cells(full):
    wl, G, pos, keep = full["wl"], full["G"], full["pos"], full["keep"]
    rng = np.random.default_rng(42)
    # the densest cells, cells where the coverage ends, and random cells anywhere
    kp = pos[keep]
    counts = np.bincount(kp[:, 1].astype(np.int64) * wl.nx + kp[:, 0], minlength=wl.nx * wl.ny)
    dense = np.argsort(counts)[-60:]
    r = np.hypot(kp[:, 0] - wl.nx / 2, kp[:, 1] - wl.ny / 2)
    edge = kp[np.argsort(r)[-60:], :2]
    rnd = rng.integers(0, [wl.nx, wl.ny], size=(80, 2))
    cells = np.concatenate([np.stack([dense % wl.nx, dense // wl.nx], 1), edge, rnd]).astype(np.int64)
    ref = orc.grid_cells(pos, keep, full["vis"], cells, wl.nx, wl.W, wl.O)
    got = G[:, cells[:, 1], cells[:, 0]]
    assert nl2(got, ref) <= TOL
    # cells no visibility reaches are exactly zero
    far = np.array([[0, 0], [wl.nx - 1, wl.ny - 1], [0, wl.ny - 1], [wl.nx - 1, 0]])
    assert np.all(orc.grid_cells(pos, keep, full["vis"], far, wl.nx, wl.W, wl.O) == 0)
    assert np.all(G[:, far[:, 1], far[:, 0]] == 0)


def test_full_size_image_of_the_grid(full):
    ref = orc.image(full["G"], W=7, correct=False)
    assert nl2(full["img"], ref) <= TOL


def test_full_size_degrid_sampled_visibilities(full):
    wl, G, pos, keep = full["wl"], full["G"], full["pos"], full["keep"]
    rng = np.random.default_rng(43)
    sel = rng.choice(np.flatnonzero(keep), size=2000, replace=False)
    ref = orc.degrid_groups(pos, G, sel, wl.W, wl.O)
    assert nl2(full["back"][sel], ref) <= TOL
