"""Parity at every workload's full size. The MWA-scale case runs in the launch configuration
bench.py times (512 antennas, 133,955,584 visibilities, 2048^2 x 4 grid, W = 7, O = 8,
default launch); its whole grid is too large for the oracle's scatter loop in a test, so
sampled cells and sampled visibilities are computed one by one (oracle.grid_cells,
oracle.degrid_groups) and the image of the GPU grid is checked whole against the oracle's
FFT. The kernel-stack, batched and differentiable workloads follow at their full sizes."""
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
    assert info["order"] == 3 and info["wg_waves"] == 4 and info["schedule"] == 1
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
# 512^2 ... 4096^2) in one plan. Every job's grid is checked on sampled cells, the smallest
# ones whole; the batched adjoint on sampled visibilities.

def test_full_size_batched_jobs():
    import torch
    from paper_0902_0915_amd import mwagrid
    jobs = synth.batched_jobs(device="cuda")
    assert len(jobs) == 96
    specs = [mwagrid.InstanceSpec.from_workload(j, with_ants=False) for j in jobs]
    rng = np.random.default_rng(45)
    with mwagrid.Plan(specs) as plan:
        grids = plan.grid([j.vis for j in jobs])
        back = plan.degrid(grids)
        torch.cuda.synchronize()
        smallest = set(np.argsort([j.nx * j.ny for j in jobs])[:3].tolist())
        for k, (j, G, b) in enumerate(zip(jobs, grids, back)):
            pos, keep, _ = orc.positions(j.uvw, j.freq, j.nx, j.ny, j.du, j.dv, j.W, j.O, flags=j.flags)
            Gh, V = to_host(G), to_host(j.vis)
            if k in smallest:
                assert nl2(Gh, orc.grid(pos, keep, V, j.nx, j.ny, j.W, j.O, nchan=j.nchan)) <= TOL, k
            kp = pos[keep]
            pick = kp[rng.choice(len(kp), size=min(30, len(kp)), replace=False), :2]
            cells = np.concatenate([pick, rng.integers(0, [j.nx, j.ny], size=(10, 2))]).astype(np.int64)
            ref = orc.grid_cells(pos, keep, V, cells, j.nx, j.W, j.O)
            assert nl2(Gh[:, cells[:, 1], cells[:, 0]], ref) <= TOL, k
            sel = rng.choice(np.flatnonzero(keep), size=min(200, int(keep.sum())), replace=False)
            assert nl2(to_host(b)[sel], orc.degrid_groups(pos, Gh, sel, j.W, j.O)) <= TOL, k
            assert np.all(to_host(b)[~keep] == 0), k
            if k % 24 == 23:
                print(f"[batched] {k + 1} of {len(jobs)} jobs checked", flush=True)


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
