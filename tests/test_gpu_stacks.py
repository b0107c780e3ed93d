"""GPU parity of the kernel-stack path (per-visibility complex kernels of varying support)
against the FP64 oracle's stack gridder and degridder."""
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


def _stack_wl(npol=1, seed=3002):
    return synth.beam_w_stacks(seed=seed, nant=24, nchan=2, ntime=3, n=512, O=4, nsrc=6,
                               n_agroups=2, n_wplanes=6, npol=npol)


def _oracle_pos(wl):
    half = (wl.kernel_support[wl.kernel_index] - 1) // 2
    return orc.positions(wl.uvw, wl.freq, wl.nx, wl.ny, wl.du, wl.dv, 0, wl.O, flags=wl.flags,
                         weights=None if wl.weights is None else wl.weights.astype(np.float64),
                         half=half)


def _kw(wl, gains=None):
    return dict(nchan=wl.nchan, weights=None if wl.weights is None else wl.weights.astype(np.float64),
                gains=gains, ant1=wl.ant1 if gains is not None else None,
                ant2=wl.ant2 if gains is not None else None)


@pytest.mark.parametrize("npol", [1, 2])
@pytest.mark.parametrize("tuning", [None, dict(tile=32), dict(tile=8, split=64), dict(tile=16, wg_waves=4)],
                         ids=str)
def test_stack_grid_parity(mw, npol, tuning):
    wl = _stack_wl(npol)
    rng = np.random.default_rng(npol)
    wl.weights = rng.uniform(0.5, 1.5, wl.ngroups).astype(np.float32)
    wl.flags = (rng.random(wl.ngroups) < 0.1).astype(np.uint8)
    gains = synth.random_gains(wl.nant, rng)
    pos, keep, counts = _oracle_pos(wl)
    ref = orc.grid_stack(pos, keep, wl.vis, wl.nx, wl.ny, wl.O, wl.kernel_stack,
                         wl.kernel_offset, wl.kernel_support, wl.kernel_index, **_kw(wl, gains))
    with mw.Plan(mw.InstanceSpec.from_workload(wl), tuning=tuning) as plan:
        assert np.array_equal(plan.positions(0), pos)
        got = to_host(plan.grid(to_dev(wl.vis), gains=to_dev(gains)))
        info = plan.info(0)
    assert info["variant"] == 5 and info["nkept"] == counts["kept"]
    assert nl2(got, ref) <= TOL, nl2(got, ref)


def test_stack_degrid_parity_adjoint_and_grad(mw):
    wl = _stack_wl(1, seed=3003)
    rng = np.random.default_rng(5)
    gains = synth.random_gains(wl.nant, rng)
    G = (rng.standard_normal((1, wl.ny, wl.nx)) + 1j * rng.standard_normal((1, wl.ny, wl.nx)))
    G = G.astype(np.complex64)
    pos, keep, _ = _oracle_pos(wl)
    args = (wl.O, wl.kernel_stack, wl.kernel_offset, wl.kernel_support, wl.kernel_index)
    ref = orc.degrid_stack(pos, keep, G, *args, **_kw(wl, gains))
    gamma = orc.degrid_stack(pos, keep, G, *args, **_kw(wl))
    rows = np.arange(wl.ngroups) // wl.nchan
    g = gains.astype(np.complex128)
    V = wl.vis.astype(np.complex128)
    g1, g2 = g[wl.ant1[rows]][:, None], g[wl.ant2[rows]][:, None]
    gg_ref = np.zeros(wl.nant, dtype=np.complex128)
    np.add.at(gg_ref, wl.ant1[rows], np.sum(g2 * np.conj(V) * gamma, axis=1))
    np.add.at(gg_ref, wl.ant2[rows], np.sum(g1 * V * np.conj(gamma), axis=1))
    with mw.Plan(mw.InstanceSpec.from_workload(wl)) as plan:
        vo, gg = plan.degrid(to_dev(G), gains=to_dev(gains), vis_in=to_dev(wl.vis),
                             want_grad_gains=True)
        plain = to_host(plan.degrid(to_dev(G)))
        Gx = to_host(plan.grid(to_dev(wl.vis)))
    assert nl2(to_host(vo), ref) <= TOL
    assert nl2(to_host(gg), gg_ref) <= 1e-4
    lhs = np.vdot(G.astype(np.complex128), Gx.astype(np.complex128))
    rhs = np.vdot(plain.astype(np.complex128), wl.vis.astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_stack_image_correction_refused(mw):
    wl = _stack_wl(1)
    with mw.Plan(mw.InstanceSpec.from_workload(wl)) as plan:
        z = to_dev(np.zeros((1, wl.ny, wl.nx), np.complex64))
        with pytest.raises(mw.MwError) as e:
            plan.image(z, correct=True)
        assert e.value.status == mw.MW_ERR_STATE
        plan.image(z, correct=False)  # the plain transform is allowed


def test_stack_workgroup_limit(mw):
    """The stack gridder's workgroups hold at most 8 waves (its launch bound): a plan asking
    for 16 is refused when it is built, with MW_ERR_UNSUPPORTED, not at its first launch."""
    wl = _stack_wl(1)
    with pytest.raises(mw.MwError) as e:
        mw.Plan(mw.InstanceSpec.from_workload(wl), tuning=dict(wg_waves=16))
    assert e.value.status == mw.MW_ERR_UNSUPPORTED
