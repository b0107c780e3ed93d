"""GPU parity of w-stacking (an imaging variant outside the paper) against the oracle: the
w-range keep rule (bit-exact positions and counts), the plane combination, and the whole
chain (one batched plan of w-planes -> grids -> corrected images -> combination) on a
non-coplanar MWA-shaped observation, through the C ABI."""
import math

import numpy as np
import pytest

import oracle as orc
from paper_0902_0915_amd import synth
from _util import nl2, to_dev, to_host

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def mw():
    import torch
    assert torch.cuda.is_available()
    from paper_0902_0915_amd import mwagrid
    return mwagrid


@pytest.fixture(scope="module")
def tilted():
    """64 antennas of the MWA-shaped layout, 4 channels, 4 times, phase centre 35 degrees from
    the zenith (so that w reaches a large fraction of u and v), 512^2 grid, 2 polarisations."""
    rng = np.random.default_rng(70)
    enu = synth.antenna_layout(64, 1500.0, rng, "r_inverse", min_sep_m=5.0)
    a1, a2 = synth.baselines(64)
    uvw = synth.uvw_tracks(enu, a1, a2, synth.hour_angles(4, 60.0), synth.MWA_LATITUDE + math.radians(35))
    freq = np.array([150e6, 151e6, 152e6, 153e6])
    n = 512
    du = synth.cell_size(uvw, freq, n)
    sky = synth.sky_disk(12, rng, math.radians(4.0), 0.5, 2.0)
    vis = synth.predict_numpy(uvw, freq, sky, npol=2, noise=0.05, rng=rng)
    return synth.Workload("tilted", 70, n, n, du, du, uvw, freq, 2, 7, 8, np.tile(a1, 4), np.tile(a2, 4), 64,
                          vis=vis)


def test_w_range_positions_and_counts(mw, tilted):
    from paper_0902_0915_amd.mwagrid import wstack_specs
    spec = mw.InstanceSpec.from_workload(tilted, with_ants=False)
    planes = wstack_specs(spec, 5)
    with mw.Plan(planes) as plan:
        total = 0
        for k, sp in enumerate(planes):
            got = plan.positions(k)
            pos, keep, counts = orc.positions(tilted.uvw, tilted.freq, tilted.nx, tilted.ny, tilted.du, tilted.dv,
                                              7, 8, wrange=sp.wrange)
            assert np.array_equal(got, pos)
            info = plan.info(k)
            assert (info["nkept"], info["nflagged"]) == (counts["kept"], counts["flagged"])
            total += info["nkept"]
    _, keep_all, _ = orc.positions(tilted.uvw, tilted.freq, tilted.nx, tilted.ny, tilted.du, tilted.dv, 7, 8)
    assert total == keep_all.sum()


def test_combine_parity(mw, tilted):
    import dataclasses
    rng = np.random.default_rng(71)
    spec = mw.InstanceSpec.from_workload(tilted, with_ants=False)
    ws = [(-40.0, -10.0), (-10.0, 5.0), (5.0, 90.0)]
    planes = [dataclasses.replace(spec, wrange=w) for w in ws]
    imgs = (rng.standard_normal((3, 2, 512, 512)) + 1j * rng.standard_normal((3, 2, 512, 512))).astype(np.complex64)
    with mw.Plan(planes) as plan:
        got = to_host(plan.wstack_combine([to_dev(z) for z in imgs]))
    ref = orc.wstack_combine(imgs.astype(np.complex128), np.array([0.5 * (a + b) for a, b in ws]), tilted.du,
                             tilted.dv)
    assert nl2(got, ref) <= TOL


def test_wstacked_image_chain(mw, tilted):
    from paper_0902_0915_amd.mwagrid import wstack_specs
    spec = mw.InstanceSpec.from_workload(tilted, with_ants=False)
    planes = wstack_specs(spec, 8)
    vis = to_dev(tilted.vis)
    with mw.Plan(planes) as plan:
        assert plan.info(-1)["batched"] == 1
        grids = plan.grid([vis] * len(planes))
        imgs = plan.image(grids, direction=1, correct=True)
        got = to_host(plan.wstack_combine(imgs))
        flat_imgs = [to_host(i) for i in imgs]
    refs = []
    for sp in planes:
        pos, keep, _ = orc.positions(tilted.uvw, tilted.freq, tilted.nx, tilted.ny, tilted.du, tilted.dv, 7, 8,
                                     wrange=sp.wrange)
        G = orc.grid(pos, keep, tilted.vis, tilted.nx, tilted.ny, 7, 8, nchan=tilted.nchan)
        refs.append(orc.image(G, W=7, correct=True))
    ref = orc.wstack_combine(np.array(refs), np.array([0.5 * sum(sp.wrange) for sp in planes]), tilted.du,
                             tilted.dv)
    q = slice(128, 384)
    for a, b in zip(flat_imgs, refs):
        assert nl2(a[:, q, q], b[:, q, q]) <= TOL
    assert nl2(got[:, q, q], ref[:, q, q]) <= TOL
