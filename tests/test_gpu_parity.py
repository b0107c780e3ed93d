"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Bars: plan integers bit-exact; grids, images and adjoints within normalised L2 1e-5;
gradients within 1e-4 (FP32 accumulation on the GPU). Sizes span many uv tiles and leave
ragged work items.
"""
import numpy as np
import pytest

import oracle as orc
from paper_0902_0915_amd import synth
from paper_0902_0915_amd.synth import C_LIGHT
from _util import nl2, oracle_grid, oracle_positions, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-5
GTOL = 1e-4


@pytest.fixture(scope="module")
def mw():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_0902_0915_amd import mwagrid
    return mwagrid


@pytest.fixture(scope="module")
def small_mwa():
    # scaled-down MWA-shaped array: 64 antennas, 8 channels, 2 times, 4 pols, 512^2 grid
    return synth.mwa_scale(seed=2002, nant=64, nchan=8, ntime=2, npol=4, n=512, nsrc=50)


@pytest.fixture(scope="module")
def tiny():
    return synth.tiny()


def _plan(mw, wl, tuning=None, **kw):
    return mw.Plan(mw.InstanceSpec.from_workload(wl, **kw), tuning=tuning)


def test_positions_bit_exact_tiny_and_mwa(mw, tiny, small_mwa):
    for wl in (tiny, small_mwa):
        with _plan(mw, wl) as plan:
            got = plan.positions(0)
            pos, keep, counts = oracle_positions(wl)
            assert np.array_equal(got, pos)
            info = plan.info(0)
            assert info["nkept"] == counts["kept"] and info["noutside"] == counts["outside"]


@pytest.mark.parametrize("W,O", [(1, 1), (3, 3), (7, 8), (9, 16), (15, 4), (5, 2)])
def test_positions_bit_exact_rules_and_edges(mw, W, O):
    rng = np.random.default_rng(W * 100 + O)
    n = 5000
    uvw = np.stack([rng.uniform(-40, 40, n), rng.uniform(-40, 40, n), np.zeros(n)], axis=1)
    uvw[:50, 0] = np.round(uvw[:50, 0] * 2 * O) / (2 * O)  # exact ties
    uvw[50:60, 0] = np.nan
    uvw[60:70, 1] = np.inf
    freq = np.array([C_LIGHT, 1.5 * C_LIGHT])
    flags = (rng.random(2 * n) < 0.1).astype(np.uint8)
    weights = rng.uniform(0.5, 1.5, 2 * n).astype(np.float32)
    weights[::37] = 0.0
    wl = synth.Workload("edges", 0, 128, 96, 1.0, 1.25, uvw, freq, 1, W, O, flags=flags,
                        weights=weights)
    with _plan(mw, wl) as plan:
        got = plan.positions(0)
        pos, keep, counts = orc.positions(uvw, freq, 128, 96, 1.0, 1.25, W, O, flags=flags,
                                          weights=weights.astype(np.float64))
        assert np.array_equal(got, pos)
        info = plan.info(0)
        assert (info["nkept"], info["nflagged"], info["noutside"]) == (
            counts["kept"], counts["flagged"], counts["outside"])


@pytest.mark.parametrize("W,O", [(3, 4), (5, 8), (7, 8), (9, 16), (15, 2), (7, 1)])
def test_kernel_tables_match_oracle(mw, W, O):
    wl = synth.tiny(W=W, O=O)
    with _plan(mw, wl) as plan:
        tab, cx, cy = plan.tables(0)
    np.testing.assert_allclose(tab, orc.kernel_table(W, O), rtol=0, atol=2e-7)
    np.testing.assert_allclose(cx, orc.correction(wl.nx, W), rtol=3e-7, atol=1e-10)
    np.testing.assert_allclose(cy, orc.correction(wl.ny, W), rtol=3e-7, atol=1e-10)


TUNINGS = [
    None,
    dict(variant=1),
    dict(variant=1, tile=16, flush=2, order=2),
    dict(tile=16, wg_waves=4),
    dict(variant=2, tile=32, wg_waves=16, split=512),
    dict(tile=16, order=2, split=300),
    dict(variant=3, tile=32),
    dict(variant=3, tile=16, flush=2),
    dict(flush=2, split=700),
    dict(variant=2, flush=2, tile=16, wg_waves=16, order=2),
    dict(variant=4, tile=8, wg_waves=16, flush=2),
    dict(variant=4, tile=16, wg_waves=8, flush=1),
    dict(variant=4, tile=8, wg_waves=4, flush=1, split=256, order=2),
    dict(variant=4, tile=8, wg_waves=1, flush=2, split=300),
    dict(variant=4, tile=16, wg_waves=2, flush=2),
    dict(variant=4, tile=8, flush=2, schedule=3, split=512),
    dict(variant=4, tile=8, flush=2, schedule=3, wg_waves=4, split=2048),
    dict(variant=4, tile=16, flush=2, schedule=3, wg_waves=4, split=256, order=2),
    dict(variant=4, tile=8, flush=2, order=3, split=300),
    dict(variant=2, tile=16, order=3),
    dict(variant=1, tile=32, order=3, flush=2),
    dict(variant=3, tile=64, order=3),
    dict(variant=4, tile=8, flush=3),
    dict(variant=4, tile=16, flush=3, wg_waves=2),
    dict(variant=4, tile=32, flush=3, wg_waves=1, order=2),
    dict(variant=6, tile=8, flush=2),
    dict(variant=6, tile=8, flush=1, split=300),
    dict(variant=6, tile=16, wg_waves=2, flush=2, order=2, split=256),
]


@pytest.mark.parametrize("tile", [8, 16, 32])
@pytest.mark.parametrize("npol", [1, 2, 4])
@pytest.mark.parametrize("W", [3, 5, 7])
def test_owner_tiles_parity_and_reproducible(mw, W, npol, tile):
    """Flush 3: each output tile gridded by one wave from every group whose footprint reaches
    it (its own and its neighbours' groups) and written once; tiles no footprint reaches are
    written as zeros over previous contents."""
    import torch
    wl = synth.mwa_scale(seed=2030 + W, nant=40, nchan=4, ntime=2, npol=npol, n=256, nsrc=10,
                         W=W, O=8)
    ref = oracle_grid(wl, wl.vis)
    with _plan(mw, wl, tuning=dict(variant=4, tile=tile, flush=3), with_ants=False) as plan:
        info = plan.info(0)
        assert info["flush"] == 3 and info["tile"] == tile
        v = to_dev(wl.vis)
        out = torch.full((npol, wl.ny, wl.nx), 5.0 - 2.0j, dtype=torch.complex64, device="cuda")
        plan.grid(v, out=out)
        a = to_host(out)
        b = to_host(plan.grid(v))
        plan.grid(v, out=out, accumulate=True)
        c = to_host(out)
    assert np.array_equal(a, b)  # fixed order, every cell written once
    assert nl2(a, ref) <= TOL, nl2(a, ref)
    assert nl2(c, 2 * ref) <= TOL
    zero = ref == 0
    assert np.all(a[zero] == 0)


@pytest.mark.parametrize("npol", [1, 4])
def test_owner_tiles_weights_gains_flags(mw, npol):
    rng = np.random.default_rng(40 + npol)
    wl = synth.mwa_scale(seed=2031, nant=48, nchan=6, ntime=2, npol=npol, n=256, nsrc=20)
    wl.flags = (rng.random(wl.ngroups) < 0.15).astype(np.uint8)
    wl.weights = rng.uniform(0.2, 2.0, wl.ngroups).astype(np.float32)
    gains = synth.random_gains(wl.nant, rng)
    ref = oracle_grid(wl, wl.vis, weights=wl.weights.astype(np.float64), gains=gains)
    with _plan(mw, wl, tuning=dict(tile=16, flush=3)) as plan:
        got = to_host(plan.grid(to_dev(wl.vis), gains=to_dev(gains)))
        # the adjoint is unchanged by the flush
        Gy = to_dev((rng.standard_normal((npol, wl.ny, wl.nx)) + 1j).astype(np.complex64))
        back = to_host(plan.degrid(Gy))
    assert nl2(got, ref) <= TOL
    pos, keep, _ = oracle_positions(wl, weights=wl.weights.astype(np.float64))
    ref_back = orc.degrid(pos, keep, to_host(Gy), wl.W, wl.O, nchan=wl.nchan,
                          weights=wl.weights.astype(np.float64))
    assert nl2(back, ref_back) <= TOL


@pytest.mark.parametrize("npol", [1, 2, 4])
def test_block_runs_equal_wave_tiles_bitwise(mw, npol):
    """Variant 6 accumulates every (cell, py) run in the order of variant 4; its padding
    entries add exact zeros. With weights, gains and flags its grid equals variant 4's bit for
    bit (and so the oracle to the same tolerance), and it is reproducible."""
    rng = np.random.default_rng(60 + npol)
    wl = synth.mwa_scale(seed=2040 + npol, nant=48, nchan=6, ntime=2, npol=npol, n=256, nsrc=20)
    wl.flags = (rng.random(wl.ngroups) < 0.15).astype(np.uint8)
    wl.weights = rng.uniform(0.2, 2.0, wl.ngroups).astype(np.float32)
    gains = synth.random_gains(wl.nant, rng)
    v, g = to_dev(wl.vis), to_dev(gains)
    with _plan(mw, wl, tuning=dict(variant=4, tile=8, flush=2, split=700)) as p4, \
            _plan(mw, wl, tuning=dict(variant=6, tile=8, flush=2, split=700)) as p6:
        assert p6.info(0)["variant"] == 6
        a4 = to_host(p4.grid(v, gains=g))
        a6 = to_host(p6.grid(v, gains=g))
        b6 = to_host(p6.grid(v, gains=g))
    np.testing.assert_array_equal(a6, a4)
    np.testing.assert_array_equal(a6, b6)
    ref = oracle_grid(wl, wl.vis, weights=wl.weights.astype(np.float64), gains=gains)
    assert nl2(a6, ref) <= TOL


def test_wave_tiles_merge_is_bit_reproducible(mw, small_mwa):
    wl = small_mwa
    with _plan(mw, wl, tuning=dict(variant=4, tile=8, flush=2), with_ants=False) as plan:
        v = to_dev(wl.vis)
        a = to_host(plan.grid(v))
        b = to_host(plan.grid(v))
    assert np.array_equal(a, b)
    assert nl2(a, oracle_grid(wl, wl.vis)) <= TOL


@pytest.mark.parametrize("tuning", TUNINGS, ids=lambda t: "default" if t is None else
                         "-".join(f"{k}{v}" for k, v in t.items()))
def test_grid_parity_mwa_4pol(mw, small_mwa, tuning):
    wl = small_mwa
    ref = oracle_grid(wl, wl.vis)
    with _plan(mw, wl, tuning=tuning, with_ants=False) as plan:
        got = to_host(plan.grid(to_dev(wl.vis)))
        info = plan.info(0)
    assert info["nwork"] > 8
    assert nl2(got, ref) <= TOL, nl2(got, ref)


@pytest.mark.parametrize("npol", [1, 2, 4])
@pytest.mark.parametrize("W", [3, 5, 7])
@pytest.mark.parametrize("variant", [1, 2, 3, 4, 6])
def test_grid_parity_variants(mw, npol, W, variant):
    wl = synth.mwa_scale(seed=2005 + W, nant=40, nchan=4, ntime=2, npol=npol, n=256, nsrc=10,
                         W=W, O=8)
    ref = oracle_grid(wl, wl.vis)
    tile = 8 if variant in (4, 6) else (64 if npol == 1 else 32)
    with _plan(mw, wl, tuning=dict(variant=variant, tile=tile, split=500),
               with_ants=False) as plan:
        got = to_host(plan.grid(to_dev(wl.vis)))
        assert plan.info(0)["variant"] == variant
    assert nl2(got, ref) <= TOL, nl2(got, ref)


@pytest.mark.parametrize("W,O,npol", [(1, 8, 1), (1, 1, 4), (9, 8, 1), (11, 8, 2), (13, 8, 1),
                                      (15, 8, 4), (7, 1, 1), (7, 3, 4), (7, 16, 1), (5, 16, 2),
                                      (15, 16, 1), (3, 3, 2)])
def test_grid_degrid_parity_supports_and_oversampling(mw, W, O, npol):
    """Every support the ABI accepts (odd W, 1...15) and oversampling at its edges (O = 1,
    odd O = 3, O = 16: the 4-bit phase fields at their top), each on the default launch,
    grid and adjoint."""
    rng = np.random.default_rng(W * 100 + O * 10 + npol)
    wl = synth.mwa_scale(seed=2010 + W + O, nant=40, nchan=4, ntime=2, npol=npol, n=256, nsrc=10,
                         W=W, O=O)
    pos, keep, _ = oracle_positions(wl)
    assert keep.sum() > 1000
    ref = orc.grid(pos, keep, wl.vis, wl.nx, wl.ny, W, O, nchan=wl.nchan)
    Gy = (rng.standard_normal((npol, wl.ny, wl.nx)) + 1j * rng.standard_normal((npol, wl.ny, wl.nx)))
    Gy = Gy.astype(np.complex64)
    ref_back = orc.degrid(pos, keep, Gy, W, O, nchan=wl.nchan)
    with _plan(mw, wl, with_ants=False) as plan:
        got = to_host(plan.grid(to_dev(wl.vis)))
        back = to_host(plan.degrid(to_dev(Gy)))
        info = plan.info(0)
    assert nl2(got, ref) <= TOL, (info, nl2(got, ref))
    assert nl2(back, ref_back) <= TOL, (info, nl2(back, ref_back))
    assert np.all(back[~keep] == 0)


@pytest.mark.parametrize("tuning", [None, dict(tile=64, wg_waves=4), dict(variant=3),
                                    dict(flush=2), dict(variant=1)], ids=str)
def test_grid_parity_tiny_1pol(mw, tiny, tuning):
    ref = oracle_grid(tiny, tiny.vis)
    with _plan(mw, tiny, tuning=tuning) as plan:
        got = to_host(plan.grid(to_dev(tiny.vis)))
    assert nl2(got, ref) <= TOL


@pytest.mark.parametrize("tuning", [None, dict(schedule=3, split=512)], ids=str)
@pytest.mark.parametrize("npol", [1, 2])
def test_grid_parity_weights_gains_flags(mw, small_mwa, npol, tuning):
    rng = np.random.default_rng(npol)
    wl = synth.mwa_scale(seed=2003, nant=48, nchan=6, ntime=2, npol=npol, n=256, nsrc=20)
    wl.flags = (rng.random(wl.ngroups) < 0.15).astype(np.uint8)
    wl.weights = rng.uniform(0.2, 2.0, wl.ngroups).astype(np.float32)
    gains = synth.random_gains(wl.nant, rng)
    ref = oracle_grid(wl, wl.vis, weights=wl.weights.astype(np.float64), gains=gains)
    with _plan(mw, wl, tuning=tuning) as plan:
        got = to_host(plan.grid(to_dev(wl.vis), gains=to_dev(gains)))
    assert nl2(got, ref) <= TOL


def test_grid_accumulate_and_overwrite(mw, tiny):
    import torch
    ref = oracle_grid(tiny, tiny.vis)
    with _plan(mw, tiny) as plan:
        v = to_dev(tiny.vis)
        out = torch.full((1, tiny.ny, tiny.nx), 3.0 + 1.0j, dtype=torch.complex64, device="cuda")
        plan.grid(v, out=out)                   # overwrite: previous contents ignored
        assert nl2(to_host(out), ref) <= TOL
        plan.grid(v, out=out, accumulate=True)  # accumulate: twice the grid
        assert nl2(to_host(out), 2 * ref) <= TOL


@pytest.mark.parametrize("tuning", [None, dict(tile=16)], ids=str)
def test_degrid_parity_and_adjoint(mw, small_mwa, tuning):
    wl = small_mwa
    rng = np.random.default_rng(7)
    G = (rng.standard_normal((4, wl.ny, wl.nx)) + 1j * rng.standard_normal((4, wl.ny, wl.nx)))
    G = G.astype(np.complex64)
    pos, keep, _ = oracle_positions(wl)
    ref = orc.degrid(pos, keep, G, wl.W, wl.O, nchan=wl.nchan)
    with _plan(mw, wl, tuning=tuning, with_ants=False) as plan:
        got = to_host(plan.degrid(to_dev(G)))
        # FP32 adjoint identity <grid(x), y> = <x, degrid(y)>
        x = wl.vis
        Gx = to_host(plan.grid(to_dev(x)))
    assert nl2(got, ref) <= TOL
    assert np.all(got[~keep] == 0)
    lhs = np.vdot(G.astype(np.complex128), Gx.astype(np.complex128))
    rhs = np.vdot(got.astype(np.complex128), x.astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


@pytest.mark.parametrize("npol,W,weighted", [(1, 7, True), (2, 5, False), (4, 3, True), (2, 7, True), (1, 3, False)])
def test_degrid_without_gains_all_lane_layouts(mw, npol, W, weighted):
    """The gains-free degridder (one wavefront per work item, factorised gather) for every
    lane layout (1, 2 or 4 polarisations) and support, with weights and flagged groups."""
    rng = np.random.default_rng(100 * npol + W)
    wl = synth.mwa_scale(seed=2007, nant=48, nchan=8, ntime=2, npol=npol, n=256, nsrc=10, W=W, make_vis=False)
    wl.flags = (rng.random(wl.ngroups) < 0.1).astype(np.uint8)
    w64 = rng.uniform(0.5, 1.5, wl.ngroups) if weighted else None
    if weighted:
        wl.weights = w64.astype(np.float32)
    G = (rng.standard_normal((npol, wl.ny, wl.nx)) + 1j * rng.standard_normal((npol, wl.ny, wl.nx)))
    G = G.astype(np.complex64)
    pos, keep, _ = oracle_positions(wl, weights=w64)
    ref = orc.degrid(pos, keep, G, W, wl.O, nchan=wl.nchan, weights=w64)
    with _plan(mw, wl, with_ants=False) as plan:
        info = plan.info(0)
        got = to_host(plan.degrid(to_dev(G)))
    assert info["variant"] == 4
    assert nl2(got, ref) <= TOL
    assert np.all(got[~keep] == 0)


@pytest.mark.parametrize("npol,W,nant", [(2, 7, 0), (4, 7, 0), (4, 5, 0), (4, 7, 9000)])
def test_degrid_gains_and_grad_gains(mw, npol, W, nant):
    """Gains and the gains' gradient through the degridder: the per-group form (2 pols) and
    the per-run form (4 pols, supports 5 and 7). Declaring 9000 antennas (the rows use 40)
    puts the per-antenna sums in HBM instead of LDS, and builds the plan's calibration lists
    by the host path for large arrays."""
    rng = np.random.default_rng(11)
    wl = synth.mwa_scale(seed=2004, nant=40, nchan=4, ntime=2, npol=npol, n=256, nsrc=10, W=W)
    wl.weights = rng.uniform(0.5, 1.5, wl.ngroups).astype(np.float32)
    if nant:
        wl.nant = nant
    gains = synth.random_gains(wl.nant, rng)
    G = (rng.standard_normal((npol, wl.ny, wl.nx)) + 1j * rng.standard_normal((npol, wl.ny, wl.nx)))
    G = G.astype(np.complex64)
    w64 = wl.weights.astype(np.float64)
    pos, keep, _ = oracle_positions(wl, weights=w64)
    ref = orc.degrid(pos, keep, G, wl.W, wl.O, nchan=wl.nchan, weights=w64, gains=gains,
                     ant1=wl.ant1, ant2=wl.ant2)
    gamma = orc.degrid(pos, keep, G, wl.W, wl.O, nchan=wl.nchan, weights=w64)
    rows = np.arange(wl.ngroups) // wl.nchan
    g = gains.astype(np.complex128)
    V = wl.vis.astype(np.complex128)
    g1, g2 = g[wl.ant1[rows]][:, None], g[wl.ant2[rows]][:, None]
    gg_ref = np.zeros(wl.nant, dtype=np.complex128)
    np.add.at(gg_ref, wl.ant1[rows], np.sum(g2 * np.conj(V) * gamma, axis=1))
    np.add.at(gg_ref, wl.ant2[rows], np.sum(g1 * V * np.conj(gamma), axis=1))
    with _plan(mw, wl) as plan:
        vo, gg = plan.degrid(to_dev(G), gains=to_dev(gains), vis_in=to_dev(wl.vis),
                             want_grad_gains=True)
    assert nl2(to_host(vo), ref) <= TOL
    assert nl2(to_host(gg), gg_ref) <= GTOL


@pytest.mark.parametrize("ny,nx", [(256, 256), (96, 128), (90, 126)])
@pytest.mark.parametrize("correct", [False, True])
def test_image_parity_both_directions(mw, ny, nx, correct):
    rng = np.random.default_rng(nx + ny)
    wl = synth.tiny()
    wl.nx, wl.ny = nx, ny
    wl.du = synth.cell_size(wl.uvw, wl.freq, min(nx, ny))
    wl.dv = wl.du
    z = (rng.standard_normal((1, ny, nx)) + 1j * rng.standard_normal((1, ny, nx))).astype(np.complex64)
    with _plan(mw, wl) as plan:
        fwd = to_host(plan.image(to_dev(z), direction=1, correct=correct))
        adj = to_host(plan.image(to_dev(z), direction=-1, correct=correct))
        zd = to_dev(z)
        plan.image(zd, direction=1, correct=correct, out=zd)  # in place
        inplace = to_host(zd)
    assert nl2(fwd, orc.image(z, W=7, correct=correct)) <= TOL
    assert nl2(adj, orc.image_adjoint(z, W=7, correct=correct)) <= TOL
    assert np.array_equal(inplace, fwd)


@pytest.mark.parametrize("ny,nx,npol", [(64, 4096, 1), (4096, 64, 1), (512, 256, 2), (2048, 2048, 4)])
def test_image_two_pass_transform_shapes(mw, ny, nx, npol):
    """Power-of-two grids use the library's two-pass transform: non-square shapes at both
    ends of its size range and several polarisations, both directions, with and without
    the correction, against the oracle."""
    import dataclasses
    rng = np.random.default_rng(nx * 3 + ny + npol)
    wl = dataclasses.replace(synth.tiny(), nx=nx, ny=ny, npol=npol)
    wl.du = synth.cell_size(wl.uvw, wl.freq, min(nx, ny))
    wl.dv = wl.du
    z = (rng.standard_normal((npol, ny, nx)) + 1j * rng.standard_normal((npol, ny, nx))).astype(np.complex64)
    with _plan(mw, wl) as plan:
        for correct in (False, True):
            fwd = to_host(plan.image(to_dev(z), direction=1, correct=correct))
            adj = to_host(plan.image(to_dev(z), direction=-1, correct=correct))
            assert nl2(fwd, orc.image(z, W=7, correct=correct)) <= TOL, correct
            assert nl2(adj, orc.image_adjoint(z, W=7, correct=correct)) <= TOL, correct


def test_image_output_view_not_16_byte_aligned(mw):
    """An output view at an odd complex offset (8-byte aligned) is transformed by the
    library's other FFT path; input and output both checked against the oracle."""
    import dataclasses
    import torch
    rng = np.random.default_rng(77)
    npol, n = 2, 256
    wl = dataclasses.replace(synth.tiny(), nx=n, ny=n, npol=npol)
    z = (rng.standard_normal((npol, n, n)) + 1j * rng.standard_normal((npol, n, n))).astype(np.complex64)
    with _plan(mw, wl) as plan:
        flat = torch.zeros(npol * n * n + 1, dtype=torch.complex64, device="cuda")
        out = flat[1:].view(npol, n, n)
        assert out.data_ptr() % 16 == 8
        src = flat.clone()
        src[1:] = to_dev(z).reshape(-1)
        plan.image(src[1:].view(npol, n, n), direction=1, correct=True, out=out)
        assert nl2(to_host(out), orc.image(z, W=7, correct=True)) <= TOL
        plan.image(to_dev(z), direction=-1, correct=False, out=out)
        assert nl2(to_host(out), orc.image_adjoint(z, W=7, correct=False)) <= TOL


@pytest.mark.parametrize("correct", [False])
def test_autograd_matches_oracle_gradients(mw, correct):
    # The loss is taken on the dirty image without the correction: dividing by the kernel
    # transform (down to 3.7e-8 at the corners) would turn FP32 rounding into the dominant
    # term of the loss and, through the adjoint's second division, of its gradient.
    import torch
    from paper_0902_0915_amd.mwagrid import grid_image
    wl = synth.differentiable(nant=32, nchan=4, ntime=2, n=256, nsrc=8)
    pos, keep, _ = oracle_positions(wl)
    V = wl.vis.astype(np.complex128)
    target = orc.image(orc.grid(pos, keep, V, wl.nx, wl.ny, 7, 8, nchan=wl.nchan), W=7,
                       correct=correct)
    gains = wl.gains.astype(np.complex128)
    loss_ref, img_ref, gv_ref, gg_ref = orc.loss_and_grads(
        pos, keep, V, gains, wl.ant1, wl.ant2, target, wl.nx, wl.ny, 7, 8, nchan=wl.nchan,
        correct=correct)
    with _plan(mw, wl) as plan:
        vis = to_dev(wl.vis).requires_grad_(True)
        g = to_dev(wl.gains).requires_grad_(True)
        img = grid_image(vis, g, plan, correct=correct)
        tgt = to_dev(target.astype(np.complex64))
        loss = torch.sum(torch.abs(img - tgt) ** 2)
        loss.backward()
        assert nl2(to_host(img), img_ref) <= TOL
        assert abs(loss.item() - loss_ref) <= 1e-4 * loss_ref
        assert nl2(to_host(vis.grad), gv_ref) <= GTOL
        assert nl2(to_host(g.grad), gg_ref) <= GTOL


def test_autograd_corrected_masked_loss_matches_oracle(mw):
    """The loss on the convolution-corrected image, summed over the inner half of the field
    (where the correction amplifies rounding at most ~15-fold): the backward then divides by
    the correction in the image adjoint, which the uncorrected form never exercises."""
    import torch
    from paper_0902_0915_amd.mwagrid import grid_image
    wl = synth.differentiable(nant=32, nchan=4, ntime=2, n=256, nsrc=8)
    pos, keep, _ = oracle_positions(wl)
    V = wl.vis.astype(np.complex128)
    target = orc.image(orc.grid(pos, keep, V, wl.nx, wl.ny, 7, 8, nchan=wl.nchan), W=7,
                       correct=True)
    mask = np.zeros((wl.ny, wl.nx))
    mask[wl.ny // 4:3 * wl.ny // 4, wl.nx // 4:3 * wl.nx // 4] = 1.0
    gains = wl.gains.astype(np.complex128)
    loss_ref, img_ref, gv_ref, gg_ref = orc.loss_and_grads(
        pos, keep, V, gains, wl.ant1, wl.ant2, target, wl.nx, wl.ny, 7, 8, nchan=wl.nchan,
        correct=True, mask=mask)
    with _plan(mw, wl) as plan:
        vis = to_dev(wl.vis).requires_grad_(True)
        g = to_dev(wl.gains).requires_grad_(True)
        img = grid_image(vis, g, plan, correct=True)
        tgt = to_dev(target.astype(np.complex64))
        m = to_dev(mask.astype(np.float32))
        loss = torch.sum(m * torch.abs(img - tgt) ** 2)
        loss.backward()
        q = slice(wl.nx // 4, 3 * wl.nx // 4)
        assert nl2(to_host(img)[q, q], img_ref[q, q]) <= TOL
        assert abs(loss.item() - loss_ref) <= 1e-4 * loss_ref
        assert nl2(to_host(vis.grad), gv_ref) <= GTOL
        assert nl2(to_host(g.grad), gg_ref) <= GTOL


def test_empty_and_fully_dropped_instances(mw):
    import torch
    freq = np.array([C_LIGHT])
    empty = synth.Workload("empty", 0, 64, 64, 1.0, 1.0, np.zeros((0, 3)), freq, 1)
    far = np.array([[500.0, 0.0, 0.0], [0.0, -900.0, 0.0]])
    outside = synth.Workload("outside", 0, 64, 64, 1.0, 1.0, far, freq, 1)
    flagged = synth.Workload("flagged", 0, 64, 64, 1.0, 1.0, np.zeros((3, 3)), freq, 1,
                             flags=np.ones(3, dtype=np.uint8))
    for wl, vis in ((empty, np.zeros((0, 1), np.complex64)), (outside, np.ones((2, 1), np.complex64)),
                    (flagged, np.ones((3, 1), np.complex64))):
        with _plan(mw, wl) as plan:
            out = torch.full((1, 64, 64), 5.0, dtype=torch.complex64, device="cuda")
            plan.grid(to_dev(vis) if len(vis) else torch.zeros((0, 1), dtype=torch.complex64,
                                                             device="cuda"), out=out)
            assert torch.count_nonzero(out).item() == 0
            info = plan.info(0)
            assert info["nkept"] == 0 and info["nwork"] == 0
            if len(vis):
                back = plan.degrid(to_dev(np.ones((1, 64, 64), np.complex64)))
                assert torch.count_nonzero(back).item() == 0


def test_state_errors_on_gpu(mw, tiny):
    with _plan(mw, tiny, with_ants=False) as plan:
        g = to_dev(np.ones(tiny.nant, np.complex64))
        with pytest.raises(mw.MwError) as e:
            plan.grid(to_dev(tiny.vis), gains=g)
        assert e.value.status == mw.MW_ERR_STATE
        with pytest.raises(mw.MwError) as e:
            plan.image(to_dev(np.zeros((1, tiny.ny, tiny.nx), np.complex64)), direction=2)
        assert e.value.status == mw.MW_ERR_INVALID_ARG
    with pytest.raises(mw.MwError) as e:
        plan.grid(to_dev(tiny.vis))
    assert e.value.status == mw.MW_ERR_STATE
    with pytest.raises(mw.MwError) as e:
        _plan(mw, synth.mwa_scale(seed=1, nant=8, nchan=1, ntime=1, npol=4, n=64, nsrc=1),
              tuning=dict(tile=64, wg_waves=16))
    assert e.value.status == mw.MW_ERR_UNSUPPORTED


def test_autotune_and_cache(mw, small_mwa, tmp_path, monkeypatch):
    wl = small_mwa
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("MW_TUNE_CACHE", str(cache))
    ref = oracle_grid(wl, wl.vis)
    with _plan(mw, wl, tuning=dict(autotune=1), with_ants=False) as plan:
        got = to_host(plan.grid(to_dev(wl.vis)))
        chosen = plan.info(0)
    assert nl2(got, ref) <= TOL
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and '"key": "gfx950' in lines[0]
    # a second plan takes the cached launch without searching again
    with _plan(mw, wl, tuning=dict(autotune=1), with_ants=False) as plan2:
        again = plan2.info(0)
        got2 = to_host(plan2.grid(to_dev(wl.vis)))
    assert len(cache.read_text().strip().splitlines()) == 1
    for k in ("tile", "split", "wg_waves", "variant", "flush", "schedule"):
        assert again[k] == chosen[k]
    assert nl2(got2, ref) <= TOL


def test_kernel_timing(mw, small_mwa):
    wl = small_mwa
    with _plan(mw, wl, with_ants=False) as plan:
        with pytest.raises(mw.MwError):
            plan.kernel_ms(0)
        plan.set_timing(True)
        plan.grid(to_dev(wl.vis))
        g, m = plan.kernel_ms(0)
        assert g > 0.0 and m > 0.0
        plan.set_timing(False)
