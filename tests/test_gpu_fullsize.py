"""Parity at every workload's full size. The MWA-scale case runs in the launch configuration
bench.py times (512 antennas, 133,955,584 visibilities, 2048^2 x 4 grid, W = 7, O = 8,
default launch) and is compared whole against the oracle's multi-threaded loops: the grid
region by region (the densest 1 % of covered cells, the rest of the coverage, and the cells
no footprint covers, which must be exactly zero), the adjoint on every visibility, and the
image of the GPU grid against the oracle's FFT. The kernel-stack, batched (every job whole)
and differentiable workloads follow at their full sizes."""
import numpy as np
import pytest

import oracle as orc
from paper_0902_0915_amd import synth
from _util import coverage, nl2, region_errors, to_host

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
    # the block-padded gridder (variant 6) on the same data, for a bitwise comparison
    with mwagrid.Plan(spec, tuning=dict(variant=6, tile=8, flush=2)) as plan6:
        out["info6"] = plan6.info(0)
        out["G6"] = to_host(plan6.grid(wl.vis))
    out["vis"] = wl.vis.cpu().numpy()
    out["wl"] = wl
    pos, keep, counts = orc.positions(wl.uvw, wl.freq, wl.nx, wl.ny, wl.du, wl.dv, wl.W, wl.O)
    out.update(pos=pos, keep=keep, counts=counts)
    return out


def test_full_size_launch_is_the_benchmarked_one(full):
    info = full["info"]
    assert info["ngroups"] == 33_488_896 and full["vis"].shape == (33_488_896, 4)
    assert info["variant"] == 4 and info["flush"] == 2 and info["tile"] == 8
    assert info["order"] == 3 and info["wg_waves"] == 4 and info["schedule"] == 1
    assert info["nkept"] == int(full["keep"].sum())


def test_full_size_grid_whole_by_region(full):
    wl, G, pos, keep = full["wl"], full["G"], full["pos"], full["keep"]
    ref = orc.grid(pos, keep, full["vis"], wl.nx, wl.ny, wl.W, wl.O, nchan=wl.nchan)
    cover = coverage(pos, keep, wl.nx, wl.ny, wl.W)
    err = region_errors(G, ref, cover)
    print(f"[fullsize] grid nl2 by region {err}", flush=True)
    assert err["dense"] <= TOL and err["rest"] <= TOL, err
    assert err["zero_nonzero_got"] == 0 and err["zero_nonzero_ref"] == 0, err
    assert nl2(G, ref) <= TOL


def test_full_size_block_runs_equal_wave_tiles(full):
    """Variant 6 at full size: the same grid as the benchmarked launch, bit for bit."""
    assert full["info6"]["variant"] == 6 and full["info6"]["nwork"] == full["info"]["nwork"]
    np.testing.assert_array_equal(full["G6"], full["G"])


def test_full_size_image_of_the_grid(full):
    ref = orc.image(full["G"], W=7, correct=False)
    assert nl2(full["img"], ref) <= TOL


def test_full_size_degrid_whole(full):
    wl, G, pos, keep = full["wl"], full["G"], full["pos"], full["keep"]
    ref = orc.degrid(pos, keep, G, wl.W, wl.O, nchan=wl.nchan)
    back = full["back"]
    assert np.all(back[~keep] == 0)
    # the groups centred in the densest 1 % of covered cells, and the others
    cover = coverage(pos, keep, wl.nx, wl.ny, wl.W)
    thr = np.quantile(cover[cover > 0], 0.99)
    kp = np.flatnonzero(keep)
    dense = cover[pos[kp, 1], pos[kp, 0]] >= thr
    e_dense = nl2(back[kp[dense]], ref[kp[dense]])
    e_rest = nl2(back[kp[~dense]], ref[kp[~dense]])
    print(f"[fullsize] degrid nl2 dense {e_dense:.2e} ({dense.sum()} groups), "
          f"rest {e_rest:.2e} ({(~dense).sum()} groups)", flush=True)
    assert e_dense <= TOL and e_rest <= TOL
    assert nl2(back, ref) <= TOL


# ---------------------------------------------------------------------------------------------
# Kernel stacks at full size: 128 antennas x 8 channels x 16 times, 4096^2 grid, O = 4, kernels
# of support 21 ... 45 (A-term x w-plane). The oracle grids the whole of it.

def test_full_size_kernel_stacks_grid_and_adjoint():
    import torch
    from paper_0902_0915_amd import mwagrid
    wl = synth.beam_w_stacks()
    assert wl.ngroups == 1_040_384 and (wl.nx, wl.ny) == (4096, 4096)
    half = (wl.kernel_support[wl.kernel_index] - 1) // 2
    pos, keep, _ = orc.positions(wl.uvw, wl.freq, wl.nx, wl.ny, wl.du, wl.dv, 0, wl.O, flags=wl.flags,
                                 half=half)
    ref = orc.grid_stack(pos, keep, wl.vis, wl.nx, wl.ny, wl.O, wl.kernel_stack, wl.kernel_offset,
                         wl.kernel_support, wl.kernel_index, nchan=wl.nchan)
    rng = np.random.default_rng(44)
    Gy = (rng.standard_normal((1, wl.ny, wl.nx)) + 1j * rng.standard_normal((1, wl.ny, wl.nx))).astype(np.complex64)
    with mwagrid.Plan(mwagrid.InstanceSpec.from_workload(wl, with_ants=False)) as plan:
        assert plan.info(0)["variant"] == 5
        got = to_host(plan.grid(torch.from_numpy(wl.vis).cuda()))
        back = to_host(plan.degrid(torch.from_numpy(Gy).cuda()))
    assert nl2(got, ref) <= TOL
    ref_back = orc.degrid_stack(pos, keep, Gy, wl.O, wl.kernel_stack, wl.kernel_offset,
                                wl.kernel_support, wl.kernel_index, nchan=wl.nchan)
    assert nl2(back, ref_back) <= TOL


# ---------------------------------------------------------------------------------------------
# The batched workload at full size: 96 uneven 1-pol jobs (1e4 ... 2e6 kept visibilities, grids
# 512^2 ... 4096^2) in one plan. Every job's grid and adjoint are compared whole.

def test_full_size_batched_jobs():
    import torch
    from paper_0902_0915_amd import mwagrid
    jobs = synth.batched_jobs(device="cuda")
    assert len(jobs) == 96
    specs = [mwagrid.InstanceSpec.from_workload(j, with_ants=False) for j in jobs]
    worst = {"dense": 0.0, "rest": 0.0, "degrid": 0.0}
    with mwagrid.Plan(specs) as plan:
        grids = plan.grid([j.vis for j in jobs])
        back = plan.degrid(grids)
        torch.cuda.synchronize()
        for k, (j, G, b) in enumerate(zip(jobs, grids, back)):
            pos, keep, _ = orc.positions(j.uvw, j.freq, j.nx, j.ny, j.du, j.dv, j.W, j.O, flags=j.flags)
            Gh, V, bh = to_host(G), to_host(j.vis), to_host(b)
            ref = orc.grid(pos, keep, V, j.nx, j.ny, j.W, j.O, nchan=j.nchan)
            err = region_errors(Gh, ref, coverage(pos, keep, j.nx, j.ny, j.W))
            assert err["dense"] <= TOL and err["rest"] <= TOL, (k, err)
            assert err["zero_nonzero_got"] == 0, (k, err)
            ed = nl2(bh, orc.degrid(pos, keep, Gh, j.W, j.O, nchan=j.nchan))
            assert ed <= TOL, (k, ed)
            assert np.all(bh[~keep] == 0), k
            worst = {"dense": max(worst["dense"], err["dense"]), "rest": max(worst["rest"], err["rest"]),
                     "degrid": max(worst["degrid"], ed)}
            if k % 24 == 23:
                print(f"[batched] {k + 1} of {len(jobs)} jobs checked whole, worst nl2 {worst}", flush=True)


# ---------------------------------------------------------------------------------------------
# Differentiable imaging at full size: 128 antennas x 8 channels x 4 times, 1024^2 grid; the
# loss on the uncorrected dirty image and its gradients with respect to visibilities and gains.

def test_full_size_differentiable_gradients():
    import torch
    from paper_0902_0915_amd import mwagrid
    from paper_0902_0915_amd.mwagrid import grid_image
    wl = synth.differentiable()
    assert wl.ngroups == 8128 * 8 * 4 and wl.nx == 1024
    pos, keep, _ = orc.positions(wl.uvw, wl.freq, wl.nx, wl.ny, wl.du, wl.dv, wl.W, wl.O, flags=wl.flags)
    V = wl.vis.astype(np.complex128)
    target = orc.image(orc.grid(pos, keep, V, wl.nx, wl.ny, wl.W, wl.O, nchan=wl.nchan), W=wl.W, correct=False)
    gains = wl.gains.astype(np.complex128)
    loss_ref, img_ref, gv_ref, gg_ref = orc.loss_and_grads(
        pos, keep, V, gains, wl.ant1, wl.ant2, target, wl.nx, wl.ny, wl.W, wl.O, nchan=wl.nchan,
        correct=False)
    with mwagrid.Plan(mwagrid.InstanceSpec.from_workload(wl)) as plan:
        vis = torch.from_numpy(wl.vis).cuda().requires_grad_(True)
        g = torch.from_numpy(wl.gains.astype(np.complex64)).cuda().requires_grad_(True)
        img = grid_image(vis, g, plan, correct=False)
        loss = torch.sum(torch.abs(img - torch.from_numpy(target.astype(np.complex64)).cuda()) ** 2)
        loss.backward()
        assert nl2(to_host(img), img_ref) <= TOL
        assert abs(loss.item() - loss_ref) <= 1e-4 * loss_ref
        assert nl2(to_host(vis.grad), gv_ref) <= 1e-4
        assert nl2(to_host(g.grad), gg_ref) <= 1e-4


def test_full_size_differentiable_corrected_masked_gradients():
    """The same workload with the loss on the corrected image over the inner half of the
    field (amplification of rounding by the correction at most ~15 there)."""
    import torch
    from paper_0902_0915_amd import mwagrid
    from paper_0902_0915_amd.mwagrid import grid_image
    wl = synth.differentiable()
    pos, keep, _ = orc.positions(wl.uvw, wl.freq, wl.nx, wl.ny, wl.du, wl.dv, wl.W, wl.O, flags=wl.flags)
    V = wl.vis.astype(np.complex128)
    target = orc.image(orc.grid(pos, keep, V, wl.nx, wl.ny, wl.W, wl.O, nchan=wl.nchan), W=wl.W, correct=True)
    mask = np.zeros((wl.ny, wl.nx))
    mask[wl.ny // 4:3 * wl.ny // 4, wl.nx // 4:3 * wl.nx // 4] = 1.0
    gains = wl.gains.astype(np.complex128)
    loss_ref, _, gv_ref, gg_ref = orc.loss_and_grads(
        pos, keep, V, gains, wl.ant1, wl.ant2, target, wl.nx, wl.ny, wl.W, wl.O, nchan=wl.nchan,
        correct=True, mask=mask)
    with mwagrid.Plan(mwagrid.InstanceSpec.from_workload(wl)) as plan:
        vis = torch.from_numpy(wl.vis).cuda().requires_grad_(True)
        g = torch.from_numpy(wl.gains.astype(np.complex64)).cuda().requires_grad_(True)
        img = grid_image(vis, g, plan, correct=True)
        m = torch.from_numpy(mask.astype(np.float32)).cuda()
        loss = torch.sum(m * torch.abs(img - torch.from_numpy(target.astype(np.complex64)).cuda()) ** 2)
        loss.backward()
        assert abs(loss.item() - loss_ref) <= 1e-4 * loss_ref
        assert nl2(to_host(vis.grad), gv_ref) <= 1e-4
        assert nl2(to_host(g.grad), gg_ref) <= 1e-4
