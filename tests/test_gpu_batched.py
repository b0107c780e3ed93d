"""GPU parity of the batched (multi-instance, persistent, graph-replayed) form."""
import os

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
def jobs():
    return synth.batched_jobs(seed=4002, njobs=7, nmin=2000, nmax=30000, sizes=(256, 512),
                              nant=64, nchan=8, ntime=2)


def _specs(mw, jobs, with_ants=True):
    return [mw.InstanceSpec.from_workload(j, with_ants=with_ants) for j in jobs]


def _oracle_grid(j, vis, gains=None):
    pos, keep, _ = orc.positions(j.uvw, j.freq, j.nx, j.ny, j.du, j.dv, j.W, j.O, flags=j.flags)
    return orc.grid(pos, keep, vis, j.nx, j.ny, j.W, j.O, nchan=j.nchan, gains=gains,
                    ant1=j.ant1 if gains is not None else None,
                    ant2=j.ant2 if gains is not None else None), pos, keep


def test_batched_grid_parity_and_graph_replays(mw, jobs):
    import torch
    rng = np.random.default_rng(1)
    refs = [_oracle_grid(j, j.vis)[0] for j in jobs]
    with mw.Plan(_specs(mw, jobs, with_ants=False)) as plan:
        vis = [to_dev(j.vis) for j in jobs]
        for rep in range(3):
            # fresh output buffers each time: the descriptor table must follow them
            out = plan.grid(vis)
            torch.cuda.synchronize()
            for j, o, r in zip(jobs, out, refs):
                assert nl2(to_host(o), r) <= TOL, (rep, j.name)
            # eager work between replays
            junk = torch.randn(1 << 20, device="cuda") * 3.0
            junk.sum().item()
        # scaled visibilities through the same graph
        vis2 = [v * 2.0 for v in vis]
        out = plan.grid(vis2)
        for o, r in zip(out, refs):
            assert nl2(to_host(o), 2 * r) <= TOL
        # accumulate into existing grids
        plan.grid(vis, out=out, accumulate=True)
        for o, r in zip(out, refs):
            assert nl2(to_host(o), 3 * r) <= TOL
        info = plan.info(-1)
    assert info["nkept"] == sum(int(_oracle_grid(j, j.vis)[2].sum()) for j in jobs)


def test_batched_grid_matches_single_instance_plans(mw, jobs):
    with mw.Plan(_specs(mw, jobs, with_ants=False)) as plan:
        batched = [to_host(g) for g in plan.grid([to_dev(j.vis) for j in jobs])]
        tiles = [plan.info(k)["tile"] for k in range(len(jobs))]
        flushes = [plan.info(k)["flush"] for k in range(len(jobs))]
        assert plan.info(-1)["batched"] == 1
    # these jobs are sparse (a few groups per 8 x 8 tile): the batch takes 16 x 16 tiles, and
    # every output tile receives few groups, so each instance takes the owner-tile flush
    assert set(tiles) == {16}
    assert set(flushes) == {3}
    for j, b, t, f in zip(jobs, batched, tiles, flushes):
        with mw.Plan(mw.InstanceSpec.from_workload(j, with_ants=False), tuning=dict(tile=t, flush=f)) as single:
            s = to_host(single.grid(to_dev(j.vis)))
        np.testing.assert_array_equal(s, b)  # identical arithmetic, identical order


def test_batch_mixes_owner_tiles_and_merge(mw):
    """A dense instance (more groups per output tile than the owner-tile cap) keeps the merge
    flush while the sparse ones in the same batch take owner tiles; both kinds run in the same
    launches, accumulate, and match the oracle and single-instance plans bit for bit."""
    import torch
    dense = synth.batched_jobs(seed=4005, njobs=1, nmin=400000, nmax=400001, sizes=(256,), nant=128,
                               nchan=8, ntime=8)
    sparse = synth.batched_jobs(seed=4006, njobs=3, nmin=3000, nmax=20000, sizes=(512, 1024),
                                nant=64, nchan=8, ntime=2)
    jobs = sparse[:2] + dense + sparse[2:]
    with mw.Plan(_specs(mw, jobs, with_ants=False), tuning=dict(tile=16)) as plan:
        flushes = [plan.info(k)["flush"] for k in range(len(jobs))]
        assert plan.info(-1)["batched"] == 1
        outs = [torch.full((1, j.ny, j.nx), 1.0 + 1.0j, dtype=torch.complex64, device="cuda") for j in jobs]
        plan.grid([to_dev(j.vis) for j in jobs], out=outs)
        got = [to_host(o) for o in outs]
        plan.grid([to_dev(j.vis) for j in jobs], out=outs, accumulate=True)
        got2 = [to_host(o) for o in outs]
    assert flushes == [3, 3, 2, 3], flushes
    for j, g, g2, f in zip(jobs, got, got2, flushes):
        ref = _oracle_grid(j, j.vis)[0]
        assert nl2(g, ref) <= TOL and nl2(g2, 2 * ref) <= TOL
        with mw.Plan(mw.InstanceSpec.from_workload(j, with_ants=False), tuning=dict(tile=16, flush=f)) as single:
            np.testing.assert_array_equal(to_host(single.grid(to_dev(j.vis))), g)


def test_dense_batch_keeps_8x8_tiles_and_a_set_tile_is_kept(mw):
    dense = synth.batched_jobs(seed=4003, njobs=2, nmin=60000, nmax=80000, sizes=(256,), nant=64,
                               nchan=8, ntime=2)
    with mw.Plan(_specs(mw, dense, with_ants=False)) as plan:
        assert {plan.info(k)["tile"] for k in range(2)} == {8}
    sparse = synth.batched_jobs(seed=4002, njobs=3, nmin=2000, nmax=30000, sizes=(512,), nant=64,
                                nchan=8, ntime=2)
    with mw.Plan(_specs(mw, sparse, with_ants=False), tuning=dict(tile=8)) as plan:
        assert {plan.info(k)["tile"] for k in range(3)} == {8}


def test_batched_degrid_with_gains_and_grad(mw, jobs):
    rng = np.random.default_rng(2)
    gains = [synth.random_gains(j.nant, rng) for j in jobs]
    Gs = [(rng.standard_normal((1, j.ny, j.nx)) + 1j * rng.standard_normal((1, j.ny, j.nx)))
          .astype(np.complex64) for j in jobs]
    with mw.Plan(_specs(mw, jobs)) as plan:
        for rep in range(2):
            vo, gg = plan.degrid([to_dev(G) for G in Gs], gains=[to_dev(g) for g in gains],
                                 vis_in=[to_dev(j.vis) for j in jobs], want_grad_gains=True)
            for j, G, g, v, gr in zip(jobs, Gs, gains, vo, gg):
                pos, keep, _ = orc.positions(j.uvw, j.freq, j.nx, j.ny, j.du, j.dv, j.W, j.O,
                                             flags=j.flags)
                ref = orc.degrid(pos, keep, G, j.W, j.O, nchan=j.nchan, gains=g, ant1=j.ant1,
                                 ant2=j.ant2)
                gamma = orc.degrid(pos, keep, G, j.W, j.O, nchan=j.nchan)
                rows = np.arange(j.ngroups) // j.nchan
                gc = g.astype(np.complex128)
                V = j.vis.astype(np.complex128)
                g1, g2 = gc[j.ant1[rows]][:, None], gc[j.ant2[rows]][:, None]
                gg_ref = np.zeros(j.nant, dtype=np.complex128)
                np.add.at(gg_ref, j.ant1[rows], np.sum(g2 * np.conj(V) * gamma, axis=1))
                np.add.at(gg_ref, j.ant2[rows], np.sum(g1 * V * np.conj(gamma), axis=1))
                got = to_host(v)
                assert nl2(got, ref) <= TOL
                assert np.all(got[~keep] == 0)
                assert nl2(to_host(gr), gg_ref) <= 1e-4


def test_batched_without_graph(mw, jobs, monkeypatch):
    monkeypatch.setenv("MW_NO_GRAPH", "1")
    with mw.Plan(_specs(mw, jobs[:3], with_ants=False)) as plan:
        out = plan.grid([to_dev(j.vis) for j in jobs[:3]])
    for j, o in zip(jobs[:3], out):
        assert nl2(to_host(o), _oracle_grid(j, j.vis)[0]) <= TOL


def test_mixed_instances_fall_back_to_per_instance_launches(mw, jobs):
    a, b = jobs[0], jobs[1]
    b5 = synth.Workload(b.name, b.seed, b.nx, b.ny, b.du, b.dv, b.uvw, b.freq, 1, 5, b.O,
                        flags=b.flags, vis=b.vis)
    with mw.Plan([mw.InstanceSpec.from_workload(a, with_ants=False),
                  mw.InstanceSpec.from_workload(b5, with_ants=False)]) as plan:
        out = plan.grid([to_dev(a.vis), to_dev(b5.vis)])
        assert plan.info(-1)["batched"] == 0
    assert nl2(to_host(out[0]), _oracle_grid(a, a.vis)[0]) <= TOL
    assert nl2(to_host(out[1]), _oracle_grid(b5, b5.vis)[0]) <= TOL


def test_autotune_tunes_the_batch_as_a_whole(mw, jobs, tmp_path, monkeypatch):
    """autotune on a multi-instance plan times the batched sequence itself: every instance
    takes the same launch, the plan stays batched, and the grids match the oracle. A cached
    result is taken by the next plan over the same jobs without a new search."""
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("MW_TUNE_CACHE", str(cache))
    refs = [_oracle_grid(j, j.vis)[0] for j in jobs]
    with mw.Plan(_specs(mw, jobs, with_ants=False), tuning=dict(autotune=1)) as plan:
        assert plan.info(-1)["batched"] == 1
        launches = {tuple(plan.info(k)[f] for f in ("tile", "wg_waves", "variant", "flush", "schedule"))
                    for k in range(len(jobs))}
        out = plan.grid([to_dev(j.vis) for j in jobs])
        back = plan.degrid(out)
    assert len(launches) == 1
    assert next(iter(launches))[3] in (2, 3)  # a bit-reproducible flush (merge or owner tiles)
    for j, o, b, r in zip(jobs, out, back, refs):
        assert nl2(to_host(o), r) <= TOL
        pos, keep, _ = orc.positions(j.uvw, j.freq, j.nx, j.ny, j.du, j.dv, j.W, j.O, flags=j.flags)
        assert nl2(to_host(b), orc.degrid(pos, keep, to_host(o), j.W, j.O, nchan=j.nchan)) <= TOL
    lines = cache.read_text().strip().splitlines()
    assert len(lines) == 1 and "/batch7/" in lines[0]
    with mw.Plan(_specs(mw, jobs, with_ants=False), tuning=dict(autotune=1)) as plan2:
        assert plan2.info(-1)["batched"] == 1
        again = {tuple(plan2.info(k)[f] for f in ("tile", "wg_waves", "variant", "flush", "schedule"))
                 for k in range(len(jobs))}
        out2 = plan2.grid([to_dev(j.vis) for j in jobs])
    assert again == launches
    assert len(cache.read_text().strip().splitlines()) == 1
    for o, r in zip(out2, refs):
        assert nl2(to_host(o), r) <= TOL


def test_plain_batch_reports_batched(mw, jobs):
    with mw.Plan(_specs(mw, jobs[:3], with_ants=False)) as plan:
        assert plan.info(-1)["batched"] == 1
