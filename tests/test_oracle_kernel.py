"""Pins for the oracle's kernel: psi_0, the oversampled tap table and the grid correction.

Each check compares the oracle with something it does not compute itself: scipy's
independent prolate-function routine, the finite-Fourier-transform eigen-property evaluated
by quadrature, or a direct numerical Fourier transform of the continuous kernel.
"""
import math

import numpy as np
import pytest
import scipy.special as sps
from numpy.polynomial.legendre import leggauss

from oracle import pswf


def _scipy_ratio(c, eta):
    eta = np.atleast_1d(eta)
    vals = np.array([sps.pro_ang1(0, 0, c, e)[0] for e in eta])
    return vals / sps.pro_ang1(0, 0, c, 0.0)[0]


@pytest.mark.parametrize("W", [3, 5, 7, 9, 11])
def test_psi0_matches_scipy(W):
    # scipy returns NaN at |eta| = 1, so stay inside.
    c = pswf.kernel_shape(W)
    eta = np.linspace(-0.995, 0.995, 41)
    mine = pswf.psi0(c, eta) / pswf.psi0(c, 0.0)
    np.testing.assert_allclose(mine, _scipy_ratio(c, eta), rtol=0, atol=1e-11)


@pytest.mark.parametrize("W", [5, 7, 9])
def test_psi0_is_eigenfunction_of_finite_fourier_transform(W):
    # int_{-1}^{1} exp(i c eta xi) psi_0(xi) dxi = lambda_0 psi_0(eta) for one real constant.
    c = pswf.kernel_shape(W)
    xi, wq = leggauss(200)
    psi_xi = pswf.psi0(c, xi)
    eta = np.linspace(-1.0, 1.0, 33)
    lhs = np.array([np.sum(wq * np.exp(1j * c * e * xi) * psi_xi) for e in eta])
    lam = lhs / pswf.psi0(c, eta)
    assert np.max(np.abs(lam.imag)) < 1e-10 * abs(lam[16])
    np.testing.assert_allclose(lam.real, lam.real[16], rtol=1e-9)


@pytest.mark.parametrize("W,O", [(7, 8), (5, 4), (7, 1), (9, 16), (7, 3)])
def test_tap_table_is_sampled_prolate_kernel(W, O):
    # Row p holds C(t - p/O) for t = -h..h, normalised to unit sum; C from scipy here.
    c = pswf.kernel_shape(W)
    h = (W - 1) // 2
    table = pswf.kernel_table(W, O)
    assert table.shape == (O, W)
    np.testing.assert_allclose(table.sum(axis=1), 1.0, rtol=0, atol=1e-14)
    for row in range(O):
        p = row - O // 2
        offs = np.arange(-h, h + 1) - p / O
        eta = 2.0 * offs / W
        ref = np.where(np.abs(eta) < 0.9999, _scipy_ratio(c, np.clip(eta, -0.9999, 0.9999)), 0.0)
        inside = np.abs(eta) < 0.9999
        ratio = table[row][inside] / ref[inside]
        np.testing.assert_allclose(ratio, ratio[0], rtol=1e-10)


def test_tap_table_zero_phase_is_symmetric_and_peaked():
    t = pswf.kernel_table(7, 8)
    zero = t[4]
    np.testing.assert_allclose(zero, zero[::-1], rtol=0, atol=1e-16)
    assert np.argmax(zero) == 3
    # phase p and -p are mirror images of each other (p = 1..3)
    for p in range(1, 4):
        np.testing.assert_allclose(t[4 + p], t[4 - p][::-1], rtol=0, atol=1e-15)


@pytest.mark.parametrize("W,N", [(7, 64), (5, 32), (9, 48)])
def test_correction_is_normalised_kernel_transform(W, N):
    # C_hat(x) = int C(t) exp(-2 pi i x t) dt over |t| <= W/2, by quadrature, against the
    # closed form psi_0(c, 2x)/psi_0(c, 0) used for the correction.
    t, wq = leggauss(400)
    t = t * (W / 2.0)
    wq = wq * (W / 2.0)
    ct = pswf.kernel_continuous(W, t)
    x = (np.arange(N) - N / 2.0) / N
    ft = np.array([np.sum(wq * ct * np.exp(-2j * math.pi * xx * t)) for xx in x])
    ft0 = np.sum(wq * ct)
    np.testing.assert_allclose(ft.real / ft0, pswf.correction(N, W), rtol=1e-9, atol=1e-13)
    assert np.max(np.abs(ft.imag)) < 1e-12 * ft0


def test_correction_edge_value():
    # At x = -1/2 the correction is psi_0(c, -1)/psi_0(c, 0); for W = 7 about 1.92e-4.
    corr = pswf.correction(256, 7)
    assert corr[128] == pytest.approx(1.0, abs=1e-15)
    assert 1.8e-4 < corr[0] < 2.0e-4
