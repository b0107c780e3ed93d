"""Pin for the oracle's gradients: FP64 central finite differences of the image-domain loss
with respect to every real and imaginary part of the gains on a 16-antenna subset of the
differentiable-imaging array, and of sampled visibility entries.

Torch's convention for a real loss of complex inputs is grad = dL/dRe + i dL/dIm.
"""
import numpy as np
import pytest

from paper_0902_0915_amd import synth


@pytest.fixture(scope="module")
def subset():
    wl = synth.differentiable()
    sub = synth.subset_antennas(wl, np.arange(16))
    # a 256^2 grid with its own 80% cell size keeps every finite-difference loss cheap
    sub.nx = sub.ny = 256
    sub.du = sub.dv = synth.cell_size(sub.uvw, sub.freq, 256)
    return sub


def _image(orc, wl, pos, keep, vis, gains, correct):
    G = orc.grid(pos, keep, vis, wl.nx, wl.ny, 7, 8, nchan=wl.nchan, gains=gains, ant1=wl.ant1,
                 ant2=wl.ant2)
    return orc.image(G, W=7, correct=correct)


def _loss_diff(orc, wl, pos, keep, vp, gp, vm, gm, target, correct):
    """L(+) - L(-) for L = sum |I - T|^2, through the exact identity
    |a - T|^2 - |b - T|^2 = Re(conj(a - b) (a + b - 2T)), which avoids subtracting two large
    losses (the loss is ~1e14 here, so the plain difference loses ~6 digits)."""
    a = _image(orc, wl, pos, keep, vp, gp, correct)
    b = _image(orc, wl, pos, keep, vm, gm, correct)
    return float(np.sum((np.conj(a - b) * (a + b - 2.0 * target)).real))


@pytest.mark.parametrize("correct", [True, False], ids=["corrected", "uncorrected"])
@pytest.mark.parametrize("step,tol,vstep,vtol", [(1e-6, 2e-6, 1e-3, 1e-6),
                                                 (1e-3, 1e-8, 1.0, 1e-8)])
def test_gradients_match_central_differences(orc, subset, step, tol, vstep, vtol, correct):
    # Along any one real coordinate of one gain (no autocorrelations, so each baseline holds
    # a given antenna once) or of one visibility, the image is affine and the loss exactly
    # quadratic: central differences carry no truncation error, only rounding, which scales
    # as 1/step. The corrected image's corner pixels are amplified ~2.7e7 by the correction,
    # so at step 1e-6 rounding alone reaches ~1e-6 relative; at 1e-3 it is ~1e-9. One
    # visibility moves the image ~1e4 times less than one gain, so its steps are larger.
    # Both loss forms are pinned: on the corrected image and on the uncorrected transform
    # (the form the GPU gradient tests use), whose adjoint must then skip the correction too.
    wl = subset
    assert wl.ngroups == 120 * 8 * 4
    pos, keep, _ = orc.positions(wl.uvw, wl.freq, wl.nx, wl.ny, wl.du, wl.dv, 7, 8)
    assert keep.all()
    vis = wl.vis.astype(np.complex128)
    true_img = orc.image(orc.grid(pos, keep, vis, wl.nx, wl.ny, 7, 8, nchan=wl.nchan), W=7,
                         correct=correct)
    gains = wl.gains.astype(np.complex128)
    loss, img, grad_v, grad_g = orc.loss_and_grads(pos, keep, vis, gains, wl.ant1, wl.ant2,
                                                   true_img, wl.nx, wl.ny, 7, 8,
                                                   nchan=wl.nchan, correct=correct)
    assert loss > 0
    fd = np.zeros(len(gains), dtype=np.complex128)
    for a in range(len(gains)):
        for unit in (1.0, 1j):
            gp, gm = gains.copy(), gains.copy()
            gp[a] += step * unit
            gm[a] -= step * unit
            d = _loss_diff(orc, wl, pos, keep, vis, gp, vis, gm, true_img, correct) / (2 * step)
            fd[a] += d * unit
    scale = np.max(np.abs(grad_g))
    assert np.max(np.abs(fd - grad_g)) <= tol * scale

    rng = np.random.default_rng(0)
    idx = rng.choice(wl.ngroups, 64, replace=False)
    fdv = np.zeros(len(idx), dtype=np.complex128)
    for j, k in enumerate(idx):
        for unit in (1.0, 1j):
            vp, vm = vis.copy(), vis.copy()
            vp[k, 0] += vstep * unit
            vm[k, 0] -= vstep * unit
            d = _loss_diff(orc, wl, pos, keep, vp, gains, vm, gains, true_img,
                           correct) / (2 * vstep)
            fdv[j] += d * unit
    scale_v = np.max(np.abs(grad_v[idx, 0]))
    assert np.max(np.abs(fdv - grad_v[idx, 0])) <= vtol * scale_v


def test_loss_zero_at_truth(orc, subset):
    wl = subset
    pos, keep, _ = orc.positions(wl.uvw, wl.freq, wl.nx, wl.ny, wl.du, wl.dv, 7, 8)
    vis = wl.vis.astype(np.complex128)
    ones = np.ones(wl.nant, dtype=np.complex128)
    target = orc.image(orc.grid(pos, keep, vis, wl.nx, wl.ny, 7, 8, nchan=wl.nchan), W=7)
    loss, _, gv, gg = orc.loss_and_grads(pos, keep, vis, ones, wl.ant1, wl.ant2, target, wl.nx,
                                         wl.ny, 7, 8, nchan=wl.nchan)
    assert loss == 0.0 and np.all(gv == 0) and np.all(gg == 0)


def test_masked_corrected_loss_gradients_match_central_differences(orc, subset):
    # The corrected image restricted to the inner half of the field (where the correction
    # amplifies by at most ~15): L = sum over the mask of |I - T|^2. The mask enters the
    # gradient as 2 mask (I - T) before the adjoint; finite differences of the masked loss
    # pin that, with the same exactness argument as above (affine image, quadratic loss).
    wl = subset
    pos, keep, _ = orc.positions(wl.uvw, wl.freq, wl.nx, wl.ny, wl.du, wl.dv, 7, 8)
    vis = wl.vis.astype(np.complex128)
    target = orc.image(orc.grid(pos, keep, vis, wl.nx, wl.ny, 7, 8, nchan=wl.nchan), W=7)
    mask = np.zeros((wl.ny, wl.nx))
    mask[wl.ny // 4:3 * wl.ny // 4, wl.nx // 4:3 * wl.nx // 4] = 1.0
    gains = wl.gains.astype(np.complex128)
    loss, img, grad_v, grad_g = orc.loss_and_grads(pos, keep, vis, gains, wl.ant1, wl.ant2,
                                                   target, wl.nx, wl.ny, 7, 8, nchan=wl.nchan,
                                                   mask=mask)
    assert loss == np.sum(mask * np.abs(img - target) ** 2)

    def ldiff(vp, gp, vm, gm):
        a = _image(orc, wl, pos, keep, vp, gp, True)
        b = _image(orc, wl, pos, keep, vm, gm, True)
        return float(np.sum(mask * (np.conj(a - b) * (a + b - 2.0 * target)).real))

    step = 1e-4
    fd = np.zeros(len(gains), dtype=np.complex128)
    for a in range(len(gains)):
        for unit in (1.0, 1j):
            gp, gm = gains.copy(), gains.copy()
            gp[a] += step * unit
            gm[a] -= step * unit
            fd[a] += ldiff(vis, gp, vis, gm) / (2 * step) * unit
    assert np.max(np.abs(fd - grad_g)) <= 1e-8 * np.max(np.abs(grad_g))
    rng = np.random.default_rng(1)
    idx = rng.choice(wl.ngroups, 32, replace=False)
    for k in idx:
        for unit in (1.0, 1j):
            vp, vm = vis.copy(), vis.copy()
            vp[k, 0] += 0.1 * unit
            vm[k, 0] -= 0.1 * unit
            d = ldiff(vp, gains, vm, gains) / 0.2
            want = (grad_v[k, 0].real if unit == 1.0 else grad_v[k, 0].imag)
            assert abs(d - want) <= 1e-8 * np.max(np.abs(grad_v))
    # the mask matters: the unmasked gradient differs
    _, _, _, gg_full = orc.loss_and_grads(pos, keep, vis, gains, wl.ant1, wl.ant2, target,
                                          wl.nx, wl.ny, 7, 8, nchan=wl.nchan)
    assert np.max(np.abs(gg_full - grad_g)) > 1e-3 * np.max(np.abs(grad_g))
