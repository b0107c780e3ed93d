"""FP64 CPU oracle for convolutional gridding, imaging and their adjoints.

Test infrastructure only: only tests/, ``__graft_entry__.smoke()`` and the cpu_baseline leg
of ``bench.py`` import it. It shares no code with the HIP library (``paper_0902_0915_amd``):
its kernel comes from ``oracle.pswf`` (Legendre eigen-solution via numpy), its loops from
``oracle/oracle.c`` (plain FP64 C, built with -ffp-contract=off), its FFTs from numpy.

Each function cites the part of the paper it follows. The paper gives one sentence on the
gridding step (Section 2.1), says the images come from a Fourier transform (Section 2,
Section 2.1) and lists the steps Gridding, FFT and Convolution Correction with their timings
(Table 1); every concrete rule below is a reading of that text, listed in the design doc.

Array conventions (all numpy):
  uvw      float64 [nrow, 3] metres          freq   float64 [nchan] Hz
  vis      complex [nrow*nchan, npol]         flags  uint8/bool [nrow*nchan] or None
  weights  float [nrow*nchan] or None         gains  complex [nant] or None, ant1/ant2 [nrow]
  pos      int32 [ngroups, 4] = cx, cy, px, py (-1 where dropped), keep bool [ngroups]
  grid     complex128 [npol, ny, nx]          image  complex128 [npol, ny, nx]
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import pswf
from .pswf import correction, kernel_table, psi0  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_D = ctypes.c_double


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from .build import build
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.orc_positions.argtypes = [_I64, _I32, _P, _P, _P, _P, _I32, _I32, _D, _D, _I32, _P, _I32,
                                  _P, _P, _P]
    lib.orc_grid.argtypes = [_I64, _I32, _P, _P, _P, _P, _P, _P, _P, _I32, _I32, _I32, _I32, _I32,
                             _P, _P, _I32]
    lib.orc_degrid.argtypes = lib.orc_grid.argtypes
    lib.orc_grid_stack.argtypes = [_I64, _I32, _P, _P, _P, _P, _P, _P, _P, _I32, _I32, _I32,
                                   _I32, _P, _P, _P, _P, _P, _I32]
    lib.orc_degrid_stack.argtypes = lib.orc_grid_stack.argtypes
    for f in (lib.orc_positions, lib.orc_grid, lib.orc_degrid, lib.orc_grid_stack,
              lib.orc_degrid_stack):
        f.restype = None
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _threads(nthreads):
    if nthreads is None or nthreads <= 0:
        return max(1, len(os.sched_getaffinity(0)))
    return int(nthreads)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _cplx(a):
    """complex array -> contiguous float64 view [..., 2] (upcast to complex128 first)."""
    if a is None:
        return None
    z = np.ascontiguousarray(a, dtype=np.complex128)
    return z.view(np.float64)


# ---------------------------------------------------------------------------------------------
# Positions, quantisation, keep rule (Section 2.1 "interpolates the samples onto a regular grid")
# ---------------------------------------------------------------------------------------------
def positions(uvw, freq, nx, ny, du, dv, W, O, flags=None, weights=None, half=None, wrange=None):
    """Quantised grid position of every (row, channel) group, and the keep mask.

    u = (u_m * f)/c, x = u/du + nx/2, qx = floor(x*O + 1/2), cx = floor((qx + O/2)/O),
    px = qx - cx*O (same in y). A group is dropped if it is flagged, has zero weight, or its
    footprint [cx-h, cx+h] x [cy-h, cy+h] leaves the grid. ``half`` gives a per-group half
    support (kernel stacks); otherwise h = (W-1)/2. ``wrange`` = (wlo, whi) keeps only groups
    with wlo <= w < whi, w = (w_m * f)/c (one plane of w-stacking); the others count as
    flagged.

    Returns (pos int32 [ngroups, 4], keep bool [ngroups], counts dict).
    """
    lib = _load()
    uvw = _c(uvw, np.float64)
    freq = _c(freq, np.float64)
    nrow, nchan = uvw.shape[0], freq.shape[0]
    ng = nrow * nchan
    if wrange is not None:
        wl = ((uvw[:, 2:3] * freq[None, :]) / C_LIGHT).reshape(-1)
        out = ~((wl >= wrange[0]) & (wl < wrange[1]))
        flags = out if flags is None else (np.asarray(flags).astype(bool) | out)
    flags = _c(flags, np.uint8)
    weights = _c(weights, np.float64)
    half = _c(half, np.int32)
    for a in (flags, weights, half):
        if a is not None and a.size != ng:
            raise ValueError("per-group array has the wrong length")
    pos = np.empty((ng, 4), dtype=np.int32)
    keep = np.empty(ng, dtype=np.uint8)
    counts = np.zeros(3, dtype=np.int64)
    lib.orc_positions(nrow, nchan, _ptr(uvw), _ptr(freq), _ptr(flags), _ptr(weights), nx, ny,
                      float(du), float(dv), O, _ptr(half), (W - 1) // 2, _ptr(pos), _ptr(keep),
                      _ptr(counts))
    return pos, keep.astype(bool), {"kept": int(counts[0]), "flagged": int(counts[1]),
                                    "outside": int(counts[2])}


def _gain_args(gains, ant1, ant2):
    if gains is None:
        return None, None, None
    if ant1 is None or ant2 is None:
        raise ValueError("gains need ant1 and ant2")
    return _cplx(gains), _c(ant1, np.int32), _c(ant2, np.int32)


# ---------------------------------------------------------------------------------------------
# Gridding (Section 2.1; Table 1 "Gridding")
# ---------------------------------------------------------------------------------------------
def grid(pos, keep, vis, nx, ny, W, O, nchan=1, weights=None, gains=None, ant1=None, ant2=None,
         table=None, out=None, nthreads=None):
    """G[pol][cy+s][cx+t] += w * g1 * conj(g2) * T[py][s] * T[px][t] * V[pol] (complex128)."""
    lib = _load()
    vis2 = np.asarray(vis)
    if vis2.ndim == 1:
        vis2 = vis2[:, None]
    ng, npol = vis2.shape
    if npol > 16:
        raise ValueError("npol > 16")
    if table is None:
        table = kernel_table(W, O)
    table = _c(table, np.float64)
    pos = _c(pos, np.int32)
    keep8 = _c(keep, np.uint8)
    visd = _cplx(vis2)
    g, a1, a2 = _gain_args(gains, ant1, ant2)
    w = _c(weights, np.float64)
    if out is None:
        out = np.zeros((npol, ny, nx), dtype=np.complex128)
    assert out.dtype == np.complex128 and out.flags.c_contiguous
    lib.orc_grid(ng, npol, _ptr(pos), _ptr(keep8), _ptr(visd), _ptr(w), _ptr(g), _ptr(a1),
                 _ptr(a2), int(nchan), nx, ny, W, O, _ptr(table), _ptr(out.view(np.float64)),
                 _threads(nthreads))
    return out


def degrid(pos, keep, grid_, W, O, nchan=1, weights=None, gains=None, ant1=None, ant2=None,
           table=None, nthreads=None):
    """Adjoint of ``grid``: y[pol] = w * conj(g1) * g2 * sum_{s,t} T[py][s] T[px][t] G[...]."""
    lib = _load()
    npol, ny, nx = grid_.shape
    if table is None:
        table = kernel_table(W, O)
    table = _c(table, np.float64)
    pos = _c(pos, np.int32)
    keep8 = _c(keep, np.uint8)
    ng = pos.shape[0]
    gd = _cplx(grid_)
    g, a1, a2 = _gain_args(gains, ant1, ant2)
    w = _c(weights, np.float64)
    out = np.zeros((ng, npol), dtype=np.complex128)
    lib.orc_degrid(ng, npol, _ptr(pos), _ptr(keep8), _ptr(gd), _ptr(w), _ptr(g), _ptr(a1),
                   _ptr(a2), int(nchan), nx, ny, W, O, _ptr(table), _ptr(out.view(np.float64)),
                   _threads(nthreads))
    return out


def grid_cells(pos, keep, vis, cells, nx, W, O, weights=None, table=None):
    """Selected cells of ``grid`` (no gains), each summed directly from its definition
    (Section 2.1, the convolution onto the grid read one output at a time): for cell (x, y)
    and polarisation p, the sum over the kept groups centred at (x - t + h, y - s + h),
    0 <= s, t < W, of T[py][s] T[px][t] w V[p]. For checks at sizes where the whole grid is
    too large for the oracle; ``cells`` is int [k, 2] of (x, y). Returns complex128 [npol, k].
    """
    h = (W - 1) // 2
    T = kernel_table(W, O) if table is None else np.asarray(table, dtype=np.float64)
    pos = np.asarray(pos)
    V = np.asarray(vis, dtype=np.complex128)
    if V.ndim == 1:
        V = V[:, None]
    w_all = None if weights is None else np.asarray(weights, dtype=np.float64)
    idx = np.flatnonzero(np.asarray(keep, dtype=bool))
    key = pos[idx, 1].astype(np.int64) * nx + pos[idx, 0]
    order = np.argsort(key, kind="stable")
    idx, key = idx[order], key[order]
    out = np.zeros((V.shape[1], len(cells)), dtype=np.complex128)
    for k, (x, y) in enumerate(np.asarray(cells, dtype=np.int64)):
        for s in range(W):
            cy = y - s + h
            if cy < 0:
                continue
            for t in range(W):
                cx = x - t + h
                if cx < 0 or cx >= nx:
                    continue
                lo, hi = np.searchsorted(key, [cy * nx + cx, cy * nx + cx + 1])
                if hi == lo:
                    continue
                g = idx[lo:hi]
                taps = T[pos[g, 3] + O // 2, s] * T[pos[g, 2] + O // 2, t]
                if w_all is not None:
                    taps = taps * w_all[g]
                out[:, k] += taps @ V[g]
    return out


def degrid_groups(pos, grid_, groups, W, O, weights=None, table=None):
    """Selected kept groups of ``degrid`` (no gains), each summed directly: y[p] =
    w sum_{s,t} T[py][s] T[px][t] G[p][cy - h + s][cx - h + t]. Returns complex128
    [len(groups), npol]."""
    h = (W - 1) // 2
    T = kernel_table(W, O) if table is None else np.asarray(table, dtype=np.float64)
    G = np.asarray(grid_, dtype=np.complex128)
    pos = np.asarray(pos)
    g = np.asarray(groups, dtype=np.int64)
    cx, cy, px, py = (pos[g, i].astype(np.int64) for i in range(4))
    out = np.zeros((len(g), G.shape[0]), dtype=np.complex128)
    for s in range(W):
        for t in range(W):
            taps = T[py + O // 2, s] * T[px + O // 2, t]
            out += taps[:, None] * G[:, cy - h + s, cx - h + t].T
    if weights is not None:
        out *= np.asarray(weights, dtype=np.float64)[g][:, None]
    return out


def grid_stack(pos, keep, vis, nx, ny, O, kstack, koffset, ksupport, kidx, nchan=1,
               weights=None, gains=None, ant1=None, ant2=None, out=None, nthreads=None):
    """Kernel-stack gridding: complex tap K_k[py][px][s][t] of the group's kernel k."""
    lib = _load()
    vis2 = np.asarray(vis)
    if vis2.ndim == 1:
        vis2 = vis2[:, None]
    ng, npol = vis2.shape
    if npol > 16:
        raise ValueError("npol > 16")
    ks = _cplx(kstack)
    ko = _c(koffset, np.int64)
    ksup = _c(ksupport, np.int32)
    ki = _c(kidx, np.int32)
    g, a1, a2 = _gain_args(gains, ant1, ant2)
    w = _c(weights, np.float64)
    if out is None:
        out = np.zeros((npol, ny, nx), dtype=np.complex128)
    lib.orc_grid_stack(ng, npol, _ptr(_c(pos, np.int32)), _ptr(_c(keep, np.uint8)),
                       _ptr(_cplx(vis2)), _ptr(w), _ptr(g), _ptr(a1), _ptr(a2), int(nchan), nx,
                       ny, O, _ptr(ks), _ptr(ko), _ptr(ksup), _ptr(ki),
                       _ptr(out.view(np.float64)), _threads(nthreads))
    return out


def degrid_stack(pos, keep, grid_, O, kstack, koffset, ksupport, kidx, nchan=1, weights=None,
                 gains=None, ant1=None, ant2=None, nthreads=None):
    """Adjoint of ``grid_stack`` (conjugated taps)."""
    lib = _load()
    npol, ny, nx = grid_.shape
    pos = _c(pos, np.int32)
    ng = pos.shape[0]
    g, a1, a2 = _gain_args(gains, ant1, ant2)
    w = _c(weights, np.float64)
    out = np.zeros((ng, npol), dtype=np.complex128)
    lib.orc_degrid_stack(ng, npol, _ptr(pos), _ptr(_c(keep, np.uint8)), _ptr(_cplx(grid_)),
                         _ptr(w), _ptr(g), _ptr(a1), _ptr(a2), int(nchan), nx, ny, O,
                         _ptr(_cplx(kstack)), _ptr(_c(koffset, np.int64)),
                         _ptr(_c(ksupport, np.int32)), _ptr(_c(kidx, np.int32)),
                         _ptr(out.view(np.float64)), _threads(nthreads))
    return out


# ---------------------------------------------------------------------------------------------
# Image = FFT, and convolution correction (Section 2, Section 2.1; Table 1 "FFT",
# "Convolution Correction")
# ---------------------------------------------------------------------------------------------
def _corr2d(ny, nx, W):
    return correction(ny, W)[:, None] * correction(nx, W)[None, :]


def image(grid_, W=7, correct=True):
    """Centred, unnormalised 2-D transform with sign +i, per polarisation:

        I[p] = sum_g G[g] exp(+2 pi i (g - N/2)(p - N/2)/N)   (separately in x and y)

    then, if ``correct``, division by the normalised kernel transform at each pixel.
    """
    g = np.asarray(grid_, dtype=np.complex128)
    ny, nx = g.shape[-2:]
    img = (nx * ny) * np.fft.fftshift(np.fft.ifft2(np.fft.ifftshift(g, axes=(-2, -1)),
                                                   axes=(-2, -1)), axes=(-2, -1))
    if correct:
        img = img / _corr2d(ny, nx, W)
    return img


def image_adjoint(img, W=7, correct=True):
    """Exact adjoint of ``image``: the correction first, then the sign -i unnormalised FFT."""
    z = np.asarray(img, dtype=np.complex128)
    ny, nx = z.shape[-2:]
    if correct:
        z = z / _corr2d(ny, nx, W)
    return np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(z, axes=(-2, -1)), axes=(-2, -1)),
                           axes=(-2, -1))


# ---------------------------------------------------------------------------------------------
# Differentiable imaging: loss and gradients in torch's convention (dL/dRe + i dL/dIm).
# Calibration solves for per-antenna complex gains (Section 2); here the gains enter the
# forward model g1 * conj(g2) * V and the gradients flow back through the adjoints.
# ---------------------------------------------------------------------------------------------
def loss_and_grads(pos, keep, vis, gains, ant1, ant2, target, nx, ny, W, O, nchan=1,
                   weights=None, correct=True, nthreads=None, mask=None):
    """L = sum |image(grid(g1 conj(g2) V)) - target|^2, with dL/dV and dL/dg.

    mask: optional real [ny, nx] array of 0/1; the sum then runs over the pixels it selects
    (L = sum mask |I - target|^2).
    grad_I = 2 mask (I - target); grad_G = image_adjoint(grad_I); gamma = degrid(grad_G)
    without gains; grad_V = conj(g1) g2 gamma;
    grad_g[a] = sum_{a1 = a} g2 conj(V) gamma + sum_{a2 = a} g1 V conj(gamma) (summed over pols).
    """
    vis2 = np.asarray(vis, dtype=np.complex128)
    if vis2.ndim == 1:
        vis2 = vis2[:, None]
    gains = np.asarray(gains, dtype=np.complex128)
    ant1 = np.asarray(ant1, dtype=np.int64)
    ant2 = np.asarray(ant2, dtype=np.int64)
    G = grid(pos, keep, vis2, nx, ny, W, O, nchan=nchan, weights=weights, gains=gains,
             ant1=ant1, ant2=ant2, nthreads=nthreads)
    img = image(G, W=W, correct=correct)
    diff = img - target
    if mask is not None:
        diff = diff * np.asarray(mask, dtype=np.float64)
    loss = float(np.sum(np.abs(diff) ** 2))
    grad_img = 2.0 * diff
    grad_grid = image_adjoint(grad_img, W=W, correct=correct)
    gamma = degrid(pos, keep, grad_grid, W, O, nchan=nchan, weights=weights, nthreads=nthreads)
    rows = np.arange(vis2.shape[0]) // nchan
    g1 = gains[ant1[rows]][:, None]
    g2 = gains[ant2[rows]][:, None]
    grad_vis = np.conj(g1) * g2 * gamma
    term1 = np.sum(g2 * np.conj(vis2) * gamma, axis=1)
    term2 = np.sum(g1 * vis2 * np.conj(gamma), axis=1)
    grad_g = np.zeros(gains.shape[0], dtype=np.complex128)
    np.add.at(grad_g, ant1[rows], term1)
    np.add.at(grad_g, ant2[rows], term2)
    return loss, img, grad_vis, grad_g


# ---------------------------------------------------------------------------------------------
# Stokes conversion (Section 2.1: the instrumental-polarisation images are converted into
# Stokes parameters by a 4 x 4 matrix that depends on time and on the position on the sky
# relative to the instrument, computed for every pixel; Table 1, "Stokes Conversion").
# ---------------------------------------------------------------------------------------------
# Coherency vector (XX, XY, YX, YY) of Stokes (I, Q, U, V) for linear feeds:
# XX = I + Q, XY = U + iV, YX = U - iV, YY = I - Q.
STOKES_TO_COHERENCY = np.array([[1, 1, 0, 0],
                                [0, 0, 1, 1j],
                                [0, 0, 1, -1j],
                                [1, -1, 0, 0]], dtype=np.complex128)


def stokes(images, jones=None, pixels=None):
    """Stokes images (I, Q, U, V) from the four instrumental-polarisation transforms.

    images: complex [4, ny, nx] in the order XX, XY, YX, YY, as ``image`` returns them from
    visibilities gridded without their Hermitian mirror. The mirrored samples (conj(V) at -u;
    for a cross product XY the mirror of YX) would add the complex conjugate image, so the
    instrumental image of the full coherency is, per pixel,
        e = (2 Re XX, XY + conj(YX), YX + conj(XY), 2 Re YY).
    jones: complex [ny, nx, 2, 2] (the instrument's response J toward each pixel at the
    snapshot's time: measured coherency = J C J^H), or None for ideal feeds (J = 1).
    Per pixel the 4 x 4 matrix M = S^-1 (J^-1 kron conj(J^-1)), with S the Stokes-to-coherency
    matrix above, maps e to (I, Q, U, V). Returns float64 [4, ny, nx] (the real parts; the
    imaginary parts vanish for Hermitian e). pixels: optional int [k, 2] of (x, y); then only
    those pixels are converted and the result is float64 [4, k].
    """
    z = np.asarray(images, dtype=np.complex128)
    npol, ny, nx = z.shape
    if npol != 4:
        raise ValueError("Stokes conversion needs the 4 instrumental polarisations")
    if pixels is None:
        yy, xx = np.divmod(np.arange(ny * nx), nx)
    else:
        px = np.asarray(pixels, dtype=np.int64)
        xx, yy = px[:, 0], px[:, 1]
    Sinv = np.linalg.inv(STOKES_TO_COHERENCY)
    out = np.empty((4, len(xx)), dtype=np.complex128)
    for k, (x, y) in enumerate(zip(xx, yy)):
        c = z[:, y, x]
        e = np.array([2.0 * c[0].real, c[1] + np.conj(c[2]), c[2] + np.conj(c[1]), 2.0 * c[3].real])
        if jones is None:
            M = Sinv
        else:
            Ji = np.linalg.inv(np.asarray(jones[y, x], dtype=np.complex128))
            M = Sinv @ np.kron(Ji, np.conj(Ji))
        out[:, k] = M @ e
    return out.real if pixels is not None else out.real.reshape(4, ny, nx)


# ---------------------------------------------------------------------------------------------
# Calibration (Section 2: the complex gain of each antenna from a large linear least-squares
# fit to observed catalogue sources; Section 2.1: the data are manipulated to measure and then
# remove the contribution of catalogue sources in decreasing order of predicted flux, each
# measurement constraining the antenna gains, iteratively; Table 1, "CML").
# ---------------------------------------------------------------------------------------------
C_LIGHT = 299_792_458.0


def predict(uvw, freq, sources, npol=1):
    """Visibilities of point sources: V[g, pol] = sum_s S_s exp(-2 pi i (u l_s + v m_s +
    w (n_s - 1))), n_s = sqrt(1 - l_s^2 - m_s^2), (u, v, w) = uvw * f / c in wavelengths, for
    group g = row * nchan + chan. Unpolarised sources: every polarisation gets the same value,
    except the cross polarisations XY, YX (1 and 2 of 4), which are zero.

    sources: float [nsrc, 3] of (l, m, flux). Returns complex128 [nrow * nchan, npol].
    """
    uvw = np.asarray(uvw, dtype=np.float64)
    freq = np.asarray(freq, dtype=np.float64)
    src = np.asarray(sources, dtype=np.float64).reshape(-1, 3)
    nrow, nchan = uvw.shape[0], freq.shape[0]
    base = np.zeros((nrow, nchan), dtype=np.complex128)
    for l, m, s in src:
        n1 = np.sqrt(1.0 - l * l - m * m) - 1.0
        path = uvw[:, 0] * l + uvw[:, 1] * m + uvw[:, 2] * n1          # metres, per row
        for c in range(nchan):
            base[:, c] += s * np.exp(-2j * np.pi * path * (freq[c] / C_LIGHT))
    out = np.zeros((nrow * nchan, npol), dtype=np.complex128)
    for p in range(npol):
        if not (npol == 4 and p in (1, 2)):
            out[:, p] = base.reshape(-1)
    return out


def stefcal(vis, model, ant1, ant2, nant, nchan, g0=None, niter=10, weights=None):
    """Per-antenna complex gains g with vis ~ g[a1] conj(g[a2]) model, by the alternating
    least-squares iteration of Salvini & Wijnholds (2014, A&A 571, A97, "StEFCal").

    Every iteration solves, for each antenna p separately and with the other antennas' gains
    held at the previous iterate, the one-unknown least-squares problem over all samples that
    involve p. The data are Hermitian in the antenna pair: a sample (a1 = q, a2 = p) is
    R_qp = V with model M_qp = M, a sample (a1 = p, a2 = q) gives R_qp = conj(V) with
    M_qp = conj(M), and both read R_qp ~ z_q conj(g_p) with z_q = g_q M_qp. The solution is
    g_p = sum w z_q conj(R_qp) / sum w |z_q|^2 over all times, channels and polarisations.
    Every second iteration the new iterate is replaced by the mean of it and the previous one
    (the method's damping). An antenna with no weight keeps its gain.

    vis, model: complex [nrow * nchan, npol]; ant1, ant2: int [nrow]; weights: real
    [nrow * nchan] or None (= 1; 0 excludes a sample). Returns (g complex128 [nant],
    rel_step = ||g_i - g_(i-1)|| / ||g_i|| of the last iteration before any averaging).
    """
    V = np.asarray(vis, dtype=np.complex128)
    M = np.asarray(model, dtype=np.complex128)
    if V.ndim == 1:
        V, M = V[:, None], M[:, None]
    rows = np.arange(V.shape[0]) // nchan
    a1 = np.asarray(ant1, dtype=np.int64)[rows]
    a2 = np.asarray(ant2, dtype=np.int64)[rows]
    w = np.ones(V.shape[0]) if weights is None else np.asarray(weights, dtype=np.float64)
    g = np.ones(nant, dtype=np.complex128) if g0 is None else np.array(g0, dtype=np.complex128)
    rel = 0.0
    for it in range(1, niter + 1):
        num = np.zeros(nant, dtype=np.complex128)
        den = np.zeros(nant, dtype=np.float64)
        for p in range(V.shape[1]):
            # samples with a1 = p: R_qp = conj(V), M_qp = conj(M), z = g[a2] conj(M)
            z = g[a2] * np.conj(M[:, p])
            np.add.at(num, a1, w * z * V[:, p])            # z conj(R) = z V
            np.add.at(den, a1, w * np.abs(z) ** 2)
            # samples with a2 = p: R_qp = V, M_qp = M, z = g[a1] M
            z = g[a1] * M[:, p]
            np.add.at(num, a2, w * z * np.conj(V[:, p]))
            np.add.at(den, a2, w * np.abs(z) ** 2)
        gnew = g.copy()
        ok = den > 0
        gnew[ok] = num[ok] / den[ok]
        nrm = np.linalg.norm(gnew)
        rel = float(np.linalg.norm(gnew - g) / nrm) if nrm > 0 else 0.0
        g = 0.5 * (gnew + g) if it % 2 == 0 else gnew
    return g, rel


def peel(vis, uvw, freq, ant1, ant2, nant, sources, npol=1, niter=10, weights=None):
    """The calibration measurement loop: catalogue sources are taken in decreasing order of
    their (predicted) flux |S|, ties in catalogue order. For each: predict its visibilities,
    measure the antenna gains toward it from the current residual data (``stefcal`` from unit
    gains), and remove it: residual -= g[a1] conj(g[a2]) model.

    Returns (residual complex128 [ngroups, npol], gains complex128 [nsrc, nant] in catalogue
    order, rel_step [nsrc], order: the processing order of catalogue indices).
    """
    R = np.array(vis, dtype=np.complex128)
    if R.ndim == 1:
        R = R[:, None]
    src = np.asarray(sources, dtype=np.float64).reshape(-1, 3)
    nchan = np.asarray(freq).shape[0]
    order = sorted(range(src.shape[0]), key=lambda k: -abs(src[k, 2]))
    rows = np.arange(R.shape[0]) // nchan
    a1 = np.asarray(ant1, dtype=np.int64)[rows]
    a2 = np.asarray(ant2, dtype=np.int64)[rows]
    gains = np.zeros((src.shape[0], nant), dtype=np.complex128)
    rels = np.zeros(src.shape[0])
    for k in order:
        M = predict(uvw, freq, src[k:k + 1], npol=npol)
        g, rels[k] = stefcal(R, M, ant1, ant2, nant, nchan, niter=niter, weights=weights)
        gains[k] = g
        R = R - (g[a1] * np.conj(g[a2]))[:, None] * M
    return R, gains, rels, order


# ---------------------------------------------------------------------------------------------
# Density weighting (an imaging variant outside the paper, which grids with the data's own
# weights): uniform and Briggs robust weights from the summed weight of each grid cell.
# ---------------------------------------------------------------------------------------------
def density_weights(pos, keep, nx, ny, weights=None, mode="uniform", robust=0.0):
    """Weights after density weighting, float64 [ngroups] (0 for dropped groups).

    The density of a cell is the summed natural weight W(c) = sum w_k over the kept groups whose
    centre cell (cx, cy) is c (the visibilities as given; their Hermitian mirrors are not
    gridded, so they are not counted). Uniform: w'_k = w_k / W(c_k). Robust (Briggs 1995, with
    robustness R): f^2 = (5 * 10^-R)^2 / (sum_c W(c)^2 / sum_k w_k) and
    w'_k = w_k / (1 + W(c_k) f^2); R -> +inf tends to natural weighting, R -> -inf to uniform
    (up to a constant factor).
    """
    pos = np.asarray(pos)
    keep = np.asarray(keep, dtype=bool)
    w = np.ones(pos.shape[0]) if weights is None else np.asarray(weights, dtype=np.float64).copy()
    w = np.where(keep, w, 0.0)
    cell = np.where(keep, pos[:, 1].astype(np.int64) * nx + pos[:, 0].astype(np.int64), 0)
    W = np.zeros(nx * ny)
    for k in np.flatnonzero(keep):           # plain accumulation in input order
        W[cell[k]] += w[k]
    out = np.zeros_like(w)
    kk = keep & (w != 0)
    if mode == "uniform":
        out[kk] = w[kk] / W[cell[kk]]
    elif mode == "robust":
        f2 = (5.0 * 10.0 ** (-robust)) ** 2 / (np.sum(W * W) / np.sum(w))
        out[kk] = w[kk] / (1.0 + W[cell[kk]] * f2)
    else:
        raise ValueError(mode)
    return out


# ---------------------------------------------------------------------------------------------
# w-stacking (an imaging variant outside the paper, which treats the array as coplanar): the
# groups are split by w into planes, each gridded and imaged on its own, and the images are
# summed with the w-term phase of their plane.
# ---------------------------------------------------------------------------------------------
def wstack_combine(images, wplanes, du, dv):
    """I[p] = sum_k images_k[p] exp(+2 pi i w_k (n - 1)) at each pixel, with
    l = (x - nx/2) / (nx du), m = (y - ny/2) / (ny dv), n = sqrt(1 - l^2 - m^2) (0 outside
    the unit circle). images: complex [nplanes, npol, ny, nx]; wplanes: [nplanes] (the w of
    each plane, in wavelengths)."""
    z = np.asarray(images, dtype=np.complex128)
    nplanes, npol, ny, nx = z.shape
    l = (np.arange(nx) - nx // 2) / (nx * du)
    m = (np.arange(ny) - ny // 2) / (ny * dv)
    n = np.sqrt(np.maximum(0.0, 1.0 - l[None, :] ** 2 - m[:, None] ** 2))
    out = np.zeros((npol, ny, nx), dtype=np.complex128)
    for k in range(nplanes):
        out += z[k] * np.exp(2j * np.pi * wplanes[k] * (n - 1.0))[None]
    return out
