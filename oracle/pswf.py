"""Oracle: the zeroth prolate spheroidal wave function and the gridding kernel built on it.

Test infrastructure only. Nothing in the product library imports, links or calls this
module; only tests/, ``__graft_entry__.smoke()`` and the cpu_baseline leg of ``bench.py``
use it. It shares no code with the HIP path.

The paper states only that the visibilities undergo a convolution that interpolates them
onto a regular grid so that an FFT can be applied (Section 2.1), and that the images are
then convolution-corrected (Table 1, "Convolution Correction"). It names no kernel. The
reading taken here (kernel family, parameters, normalisation) is the prolate spheroidal
kernel of order zero with shape parameter c = pi*W/2:

    C(t) = psi_0(c, 2t/W),  |t| <= W/2   (t in grid cells)

psi_0 is computed as the lowest eigenvector of the prolate differential operator

    L psi = -d/deta[(1 - eta^2) dpsi/deta] + c^2 eta^2 psi

expanded in orthonormal Legendre polynomials. In that basis the first term is diagonal
(k(k+1)) and eta is the symmetric tridiagonal Jacobi matrix J with
J[k, k+1] = (k+1)/sqrt((2k+1)(2k+3)), so L = diag(k(k+1)) + c^2 J^2. The dense symmetric
eigenproblem is solved with numpy's ``eigh`` (a library primitive).
"""
from __future__ import annotations

import functools
import math

import numpy as np
from numpy.polynomial import legendre as _leg


@functools.lru_cache(maxsize=64)
def prolate_legendre(c: float, nterms: int | None = None):
    """Return (chi_0, b) with psi_0(c, eta) = sum_k b[k] P_k(eta) (standard Legendre P_k).

    The sign is fixed so that psi_0(c, 0) > 0. The overall scale is that of a unit-norm
    eigenvector in the orthonormal basis, i.e. int_{-1}^{1} psi_0^2 = 1.
    """
    if nterms is None:
        nterms = 2 * int(math.ceil(c)) + 60
    m = int(nterms)
    k = np.arange(m + 2, dtype=np.float64)
    kk = k[1:]
    off = kk / np.sqrt((2.0 * kk - 1.0) * (2.0 * kk + 1.0))  # J[k-1, k], k = 1..m+1
    jac = np.diag(off, 1) + np.diag(off, -1)
    op = np.diag(k * (k + 1.0)) + (c * c) * (jac @ jac)
    op = op[:m, :m]  # drop the rows where the truncated J^2 is incomplete
    vals, vecs = np.linalg.eigh(op)
    d = vecs[:, 0].copy()
    b = d * np.sqrt((2.0 * np.arange(m) + 1.0) / 2.0)
    if _leg.legval(0.0, b) < 0.0:
        b = -b
    return float(vals[0]), b


def psi0(c: float, eta) -> np.ndarray:
    """psi_0(c, eta) for |eta| <= 1 (float64)."""
    _, b = prolate_legendre(float(c))
    return _leg.legval(np.asarray(eta, dtype=np.float64), b)


def kernel_shape(W: int) -> float:
    """Shape parameter c = pi*W/2 (reading of an unspecified kernel; alpha = 0)."""
    return math.pi * W / 2.0


def kernel_continuous(W: int, t) -> np.ndarray:
    """Unnormalised continuous kernel C(t) = psi_0(c, 2t/W) on |t| <= W/2, zero outside."""
    t = np.asarray(t, dtype=np.float64)
    eta = 2.0 * t / W
    out = np.zeros_like(t)
    inside = np.abs(eta) <= 1.0
    out[inside] = psi0(kernel_shape(W), eta[inside])
    return out


def kernel_table(W: int, O: int) -> np.ndarray:
    """Oversampled tap table T[p + O//2][t + h], float64 of shape [O, W].

    A visibility whose quantised position is cell cx plus phase p/O (p in [-O//2, O - O//2))
    contributes to cell cx + t (t in [-h, h], h = (W-1)/2) with weight C(t - p/O), and each
    phase row is divided by its own sum so that every row sums to one.
    """
    if W < 1 or W % 2 == 0:
        raise ValueError("support W must be odd and positive")
    if O < 1:
        raise ValueError("oversampling O must be >= 1")
    h = (W - 1) // 2
    table = np.empty((O, W), dtype=np.float64)
    for row in range(O):
        p = row - O // 2
        offs = np.arange(-h, h + 1, dtype=np.float64) - p / O
        vals = kernel_continuous(W, offs)
        table[row] = vals / vals.sum()
    return table


def correction(N: int, W: int) -> np.ndarray:
    """Grid-correction function at the N image pixels along one axis.

    Pixel p sits at x = (p - N/2)/N in units of the field of view. The Fourier transform of
    C is proportional to psi_0(c, 2x) (the prolate functions are eigenfunctions of the
    finite Fourier transform on [-1, 1]), so the normalised transform is
    psi_0(c, 2x)/psi_0(c, 0). The image is divided by this, once per axis.
    """
    x = (np.arange(N, dtype=np.float64) - N / 2.0) / N
    c = kernel_shape(W)
    return psi0(c, 2.0 * x) / psi0(c, 0.0)
