"""GPU parity of density weighting (uniform and Briggs robust, an imaging variant beside the
paper's gridding step) against the oracle: the grid and its adjoint with the plan's density
weights, with and without given weights and flags, its independence of the order of the
GPU's atomic cell sums (two plans, identical bits), and a batched plan."""
import numpy as np
import pytest

import oracle as orc
from paper_0902_0915_amd import synth
from _util import nl2, oracle_positions, to_dev, to_host

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def mw():
    import torch
    assert torch.cuda.is_available()
    from paper_0902_0915_amd import mwagrid
    return mwagrid


def _oracle(wl, mode, robust, weights):
    pos, keep, _ = orc.positions(wl.uvw, wl.freq, wl.nx, wl.ny, wl.du, wl.dv, wl.W, wl.O, flags=wl.flags,
                                 weights=weights)
    wd = orc.density_weights(pos, keep, wl.nx, wl.ny, weights, mode, robust)
    G = orc.grid(pos, keep, wl.vis, wl.nx, wl.ny, wl.W, wl.O, nchan=wl.nchan, weights=wd)
    return pos, keep, wd, G


@pytest.mark.parametrize("mode,robust", [("uniform", 0.0), ("robust", -1.0), ("robust", 0.0), ("robust", 1.5)])
@pytest.mark.parametrize("given", [False, True])
def test_density_weighted_grid_and_adjoint(mw, mode, robust, given):
    rng = np.random.default_rng(10 + given)
    wl = synth.mwa_scale(seed=2060, nant=64, nchan=6, ntime=2, npol=2, n=256, nsrc=20)
    wl.flags = (rng.random(wl.ngroups) < 0.1).astype(np.uint8)
    weights = rng.uniform(0.3, 2.0, wl.ngroups) if given else None
    wl.weights = None if weights is None else weights.astype(np.float32)
    pos, keep, wd, G = _oracle(wl, mode, robust, None if weights is None else weights.astype(np.float32).astype(np.float64))
    spec = mw.InstanceSpec.from_workload(wl, with_ants=False)
    spec.weighting, spec.robust = mode, robust
    Gy = (rng.standard_normal((2, wl.ny, wl.nx)) + 1j * rng.standard_normal((2, wl.ny, wl.nx))).astype(np.complex64)
    with mw.Plan(spec) as plan:
        got = to_host(plan.grid(to_dev(wl.vis)))
        back = to_host(plan.degrid(to_dev(Gy)))
    assert nl2(got, G) <= TOL, nl2(got, G)
    ref_back = orc.degrid(pos, keep, Gy, wl.W, wl.O, nchan=wl.nchan, weights=wd)
    assert nl2(back, ref_back) <= TOL


def test_density_weighting_is_order_independent_and_uniform_flattens(mw):
    wl = synth.mwa_scale(seed=2061, nant=96, nchan=8, ntime=2, npol=1, n=256, nsrc=10)
    spec = mw.InstanceSpec.from_workload(wl, with_ants=False)
    spec.weighting = "uniform"
    with mw.Plan(spec) as a, mw.Plan(spec) as b:
        ga = to_host(a.grid(to_dev(wl.vis)))
        gb = to_host(b.grid(to_dev(wl.vis)))
        # gridding unit visibilities with uniform weights: each occupied cell's weights sum to
        # one, so the grid's total is the number of occupied cells
        ones = to_dev(np.ones_like(wl.vis))
        tot = to_host(a.grid(ones)).sum()
    np.testing.assert_array_equal(ga, gb)
    pos, keep, _ = oracle_positions(wl)
    occupied = np.unique(pos[keep, 1].astype(np.int64) * wl.nx + pos[keep, 0]).size
    assert abs(tot - occupied) <= 1e-4 * occupied


def test_density_weighting_in_a_batch(mw):
    jobs = synth.batched_jobs(seed=4008, njobs=4, nmin=3000, nmax=30000, sizes=(256, 512), nant=64, nchan=8,
                              ntime=2)
    specs = []
    for j in jobs:
        sp = mw.InstanceSpec.from_workload(j, with_ants=False)
        sp.weighting, sp.robust = "robust", 0.5
        specs.append(sp)
    with mw.Plan(specs) as plan:
        assert plan.info(-1)["batched"] == 1
        grids = [to_host(g) for g in plan.grid([to_dev(j.vis) for j in jobs])]
    for j, g in zip(jobs, grids):
        _, _, _, G = _oracle(j, "robust", 0.5, None)
        assert nl2(g, G) <= TOL
