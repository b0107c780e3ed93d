"""Seeded synthetic MWA-shaped inputs: array layouts, uvw tracks, skies, visibilities, flags,
gains, kernel stacks and batched job sets.

This module produces inputs only. It contains none of the gridding, imaging or adjoint
arithmetic, so both the HIP path and the FP64 oracle can take their inputs from it.

Shapes follow the paper's description of the instrument (Section 1: a 512-element array;
Section 2: about 130,000 baselines, many frequency channels, 4 polarisations) and the
workloads named in the design doc. The paper publishes no dataset or worked example; every array
here is synthetic and seeded (``seed = 1000 * config + instance``).

Conventions: rows are time-major (row = t * nbl + b); visibilities are
[row * nchan + chan, pol] complex64; u points east, v north (at hour angle 0, phase centre at
the zenith); a point source at direction cosines (l, m) contributes S exp(-2 pi i (u l + v m +
w (n - 1))).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

C_LIGHT = 299_792_458.0
OMEGA_EARTH = 7.2921159e-5  # rad/s
MWA_LATITUDE = math.radians(-26.70)


# ---------------------------------------------------------------------------------------------
# Array geometry
# ---------------------------------------------------------------------------------------------
def antenna_layout(nant, radius_m, rng, profile="uniform", min_sep_m=0.0):
    """East/north/up antenna positions [nant, 3] in a disk of the given radius.

    profile "uniform": uniform surface density (r = R sqrt(U)).
    profile "r_inverse": surface density proportional to 1/r (r = R U), centrally condensed.
    min_sep_m: resample any antenna closer than this to an earlier one.
    """
    pos = np.zeros((nant, 3))
    n = 0
    tries = 0
    while n < nant:
        tries += 1
        if tries > 1000 * nant:
            raise RuntimeError("could not place antennas with the requested minimum spacing")
        u = rng.random()
        r = radius_m * (math.sqrt(u) if profile == "uniform" else u)
        th = rng.random() * 2.0 * math.pi
        p = np.array([r * math.cos(th), r * math.sin(th), 0.0])
        if min_sep_m > 0.0 and n > 0:
            if np.min(np.hypot(pos[:n, 0] - p[0], pos[:n, 1] - p[1])) < min_sep_m:
                continue
        pos[n] = p
        n += 1
    return pos


def baselines(nant):
    """All antenna pairs i < j, in the usual order: (ant1, ant2) int32 [nant*(nant-1)/2]."""
    a1, a2 = np.triu_indices(nant, k=1)
    return a1.astype(np.int32), a2.astype(np.int32)


def enu_to_xyz(enu, lat=MWA_LATITUDE):
    e, n, u = enu[:, 0], enu[:, 1], enu[:, 2]
    x = -math.sin(lat) * n + math.cos(lat) * u
    y = e
    z = math.cos(lat) * n + math.sin(lat) * u
    return np.stack([x, y, z], axis=1)


def uvw_tracks(enu, ant1, ant2, hour_angles, dec, lat=MWA_LATITUDE):
    """uvw in metres, [ntime * nbl, 3], time-major, by the standard rotation of the
    equatorial baseline vector to the (hour angle, declination) of the phase centre."""
    xyz = enu_to_xyz(enu, lat)
    b = xyz[ant2] - xyz[ant1]
    out = np.empty((len(hour_angles), b.shape[0], 3))
    sd, cd = math.sin(dec), math.cos(dec)
    for i, H in enumerate(hour_angles):
        sh, ch = math.sin(H), math.cos(H)
        out[i, :, 0] = sh * b[:, 0] + ch * b[:, 1]
        out[i, :, 1] = -sd * ch * b[:, 0] + sd * sh * b[:, 1] + cd * b[:, 2]
        out[i, :, 2] = cd * ch * b[:, 0] - cd * sh * b[:, 1] + sd * b[:, 2]
    return out.reshape(-1, 3)


def hour_angles(ntime, cadence_s):
    return [(t - (ntime - 1) / 2.0) * cadence_s * OMEGA_EARTH for t in range(ntime)]


def cell_size(uvw, freq, n, fill=0.8):
    """Cell size [wavelengths] so that the longest |u| or |v| fills ``fill`` of the half grid."""
    umax = np.max(np.abs(uvw[:, :2])) * np.max(freq) / C_LIGHT
    return float(umax / (fill * n / 2.0))


# ---------------------------------------------------------------------------------------------
# Skies and visibilities
# ---------------------------------------------------------------------------------------------
@dataclass
class Sky:
    l: np.ndarray
    m: np.ndarray
    flux: np.ndarray


def sky_disk(nsrc, rng, radius_rad, fmin, fmax):
    """Sources uniform within an angular radius of the phase centre, flux U[fmin, fmax]."""
    r = math.sin(radius_rad) * np.sqrt(rng.random(nsrc))
    th = rng.random(nsrc) * 2.0 * math.pi
    return Sky(r * np.cos(th), r * np.sin(th), fmin + (fmax - fmin) * rng.random(nsrc))


def sky_powerlaw_box(nsrc, rng, half_width, smin, smax, slope=2.5):
    """dN/dS ~ S^-slope on [smin, smax]; (l, m) uniform in |l|, |m| <= half_width."""
    a = 1.0 - slope
    u = rng.random(nsrc)
    flux = (smin ** a + u * (smax ** a - smin ** a)) ** (1.0 / a)
    l = (2.0 * rng.random(nsrc) - 1.0) * half_width
    m = (2.0 * rng.random(nsrc) - 1.0) * half_width
    return Sky(l, m, flux)


def predict_numpy(uvw, freq, sky, npol=1, noise=0.0, rng=None, xy_noise_only=True):
    """Point-source visibilities [nrow*nchan, npol] complex64 (numpy; small inputs).

    npol == 4 gives instrumental XX, XY, YX, YY with XX = YY = sky + noise, XY = YX = noise.
    """
    nrow, nchan = uvw.shape[0], freq.shape[0]
    n = np.sqrt(np.maximum(0.0, 1.0 - sky.l ** 2 - sky.m ** 2)) - 1.0
    out = np.zeros((nrow, nchan), dtype=np.complex128)
    for ci, f in enumerate(freq):
        lam = C_LIGHT / f
        ph = -2.0 * math.pi * (np.outer(uvw[:, 0], sky.l) + np.outer(uvw[:, 1], sky.m)
                               + np.outer(uvw[:, 2], n)) / lam
        out[:, ci] = (np.exp(1j * ph) * sky.flux[None, :]).sum(axis=1)
    return _pols(out.reshape(-1), npol, noise, rng, xy_noise_only)


def _pols(base, npol, noise, rng, xy_noise_only):
    ng = base.shape[0]
    vis = np.zeros((ng, npol), dtype=np.complex128)
    for p in range(npol):
        if npol == 4 and xy_noise_only and p in (1, 2):
            continue
        vis[:, p] = base
    if noise > 0.0:
        vis += noise * (rng.standard_normal((ng, npol)) + 1j * rng.standard_normal((ng, npol)))
    return vis.astype(np.complex64)


def predict_torch(uvw, freq, sky, npol, noise, seed, device, chunk_groups=1 << 20,
                  chunk_src=128):
    """Same as ``predict_numpy`` for large inputs: FP64 phases on ``device`` (torch), chunked.

    Returns a torch complex64 tensor [nrow*nchan, npol] on ``device``. Noise is drawn from a
    torch generator seeded with ``seed`` (so values differ from the numpy path).
    """
    import torch

    dev = torch.device(device)
    nrow, nchan = uvw.shape[0], freq.shape[0]
    ng = nrow * nchan
    u = torch.as_tensor(uvw, dtype=torch.float64, device=dev)
    f = torch.as_tensor(freq, dtype=torch.float64, device=dev)
    l = torch.as_tensor(sky.l, dtype=torch.float64, device=dev)
    m = torch.as_tensor(sky.m, dtype=torch.float64, device=dev)
    s = torch.as_tensor(sky.flux, dtype=torch.float64, device=dev)
    nn = torch.sqrt(torch.clamp(1.0 - l * l - m * m, min=0.0)) - 1.0
    base = torch.empty(ng, dtype=torch.complex64, device=dev)
    rows_per = max(1, chunk_groups // nchan)
    for r0 in range(0, nrow, rows_per):
        r1 = min(nrow, r0 + rows_per)
        uu = u[r0:r1]
        acc = torch.zeros((r1 - r0) * nchan, dtype=torch.complex128, device=dev)
        scale = (f / C_LIGHT)  # [nchan]
        for s0 in range(0, l.shape[0], chunk_src):
            s1 = min(l.shape[0], s0 + chunk_src)
            # path length in metres per (row, source), then per channel in wavelengths
            d = (uu[:, 0:1] * l[None, s0:s1] + uu[:, 1:2] * m[None, s0:s1]
                 + uu[:, 2:3] * nn[None, s0:s1])  # [rows, src]
            ph = (-2.0 * math.pi) * d[:, None, :] * scale[None, :, None]  # [rows, chan, src]
            ph = torch.remainder(ph, 2.0 * math.pi)
            acc += (torch.polar(s[s0:s1].expand_as(ph), ph)).sum(dim=2).reshape(-1)
        base[r0 * nchan:r1 * nchan] = acc.to(torch.complex64)
    vis = torch.zeros((ng, npol), dtype=torch.complex64, device=dev)
    for p in range(npol):
        if npol == 4 and p in (1, 2):
            continue
        vis[:, p] = base
    if noise > 0.0:
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed)
        vis += (noise * torch.complex(torch.randn((ng, npol), generator=gen, device=dev),
                                      torch.randn((ng, npol), generator=gen, device=dev)))
    return vis


def random_gains(nant, rng, amp_sigma=0.1, phase_max=0.3):
    amp = 1.0 + amp_sigma * rng.standard_normal(nant)
    ph = rng.uniform(-phase_max, phase_max, nant)
    return (amp * np.exp(1j * ph)).astype(np.complex64)


# ---------------------------------------------------------------------------------------------
# Workload descriptions
# ---------------------------------------------------------------------------------------------
@dataclass
class Workload:
    """One gridding instance's inputs (numpy, host)."""
    name: str
    seed: int
    nx: int
    ny: int
    du: float
    dv: float
    uvw: np.ndarray            # [nrow, 3] float64 metres
    freq: np.ndarray           # [nchan] float64 Hz
    npol: int
    W: int = 7
    O: int = 8
    ant1: np.ndarray | None = None
    ant2: np.ndarray | None = None
    nant: int = 0
    flags: np.ndarray | None = None     # [nrow*nchan] uint8
    weights: np.ndarray | None = None   # [nrow*nchan] float32
    vis: np.ndarray | None = None       # [nrow*nchan, npol] complex64 (None: make later)
    sky: Sky | None = None
    noise: float = 0.0
    gains: np.ndarray | None = None
    kernel_stack: np.ndarray | None = None   # complex64 ragged
    kernel_offset: np.ndarray | None = None  # int64 [nkernel]
    kernel_support: np.ndarray | None = None  # int32 [nkernel]
    kernel_index: np.ndarray | None = None   # int32 [nrow*nchan]
    meta: dict = field(default_factory=dict)

    @property
    def nrow(self):
        return self.uvw.shape[0]

    @property
    def nchan(self):
        return self.freq.shape[0]

    @property
    def ngroups(self):
        return self.nrow * self.nchan


def tiny(seed=1001, W=7, O=8, n=256):
    """32 antennas uniform in a 1.5 km disk, 496 baselines, 1 channel at 150 MHz, 1 time step,
    1 polarisation, 5 point sources (U[0.1, 1] Jy within 10 deg) plus complex Gaussian noise
    sigma = 0.1; 256^2 grid, cell so that the longest baseline fills 80% of the half grid."""
    rng = np.random.default_rng(seed)
    enu = antenna_layout(32, 1500.0, rng, "uniform")
    a1, a2 = baselines(32)
    uvw = uvw_tracks(enu, a1, a2, [0.0], MWA_LATITUDE)
    freq = np.array([150e6])
    du = cell_size(uvw, freq, n)
    sky = sky_disk(5, rng, math.radians(10.0), 0.1, 1.0)
    vis = predict_numpy(uvw, freq, sky, npol=1, noise=0.1, rng=rng)
    return Workload("tiny", seed, n, n, du, du, uvw, freq, 1, W, O, a1, a2, 32, vis=vis,
                    sky=sky, noise=0.1)


def mwa_scale(seed=2001, nant=512, nchan=32, ntime=8, npol=4, n=2048, nsrc=1000, W=7, O=8,
              make_vis=True, device=None):
    """512 antennas, density ~ 1/r within 1.5 km (5 m minimum spacing), all 130,816 baselines
    x 32 channels (140.5 + k MHz) x 8 times (8 s cadence, earth rotation, zenith phase centre
    at hour angle 0) x 4 instrumental polarisations; 1000 point sources with dN/dS ~ S^-2.5 on
    [0.1, 10] Jy uniform in the inner 80% of the field; XX = YY = sky + noise, XY = YX = noise
    (sigma 0.1); 2048^2 grid per polarisation.

    ``nant``/``nchan``/``ntime``/``n``/``nsrc`` can be reduced for scaled-down tests.
    ``device``: torch device for the large visibility prediction (None: numpy).
    """
    rng = np.random.default_rng(seed)
    enu = antenna_layout(nant, 1500.0, rng, "r_inverse", min_sep_m=5.0)
    a1, a2 = baselines(nant)
    uvw = uvw_tracks(enu, a1, a2, hour_angles(ntime, 8.0), MWA_LATITUDE)
    freq = (140.5e6 + 1e6 * np.arange(nchan)) if nchan > 1 else np.array([150e6])
    du = cell_size(uvw, freq, n)
    half = 0.4 / du  # inner 80% of the field of view (1/du wide)
    sky = sky_powerlaw_box(nsrc, rng, half, 0.1, 10.0)
    wl = Workload("mwa_scale", seed, n, n, du, du, uvw, freq, npol, W, O,
                  np.tile(a1, ntime), np.tile(a2, ntime), nant, sky=sky, noise=0.1)
    wl.meta.update(nbl=len(a1), ntime=ntime)
    if make_vis:
        if device is None:
            wl.vis = predict_numpy(uvw, freq, sky, npol=npol, noise=0.1, rng=rng)
        else:
            wl.vis = predict_torch(uvw, freq, sky, npol, 0.1, seed, device)
    return wl


def differentiable(seed=5001, nant=128, nchan=8, ntime=4, n=1024, nsrc=20, W=7, O=8):
    """128 antennas (8128 baselines) x 8 channels x 4 times x 1 polarisation, 1024^2 grid,
    a 20-source sky, true gains with amplitude 1 + 0.1 N(0,1) and phase U[-0.3, 0.3] rad."""
    rng = np.random.default_rng(seed)
    enu = antenna_layout(nant, 1500.0, rng, "r_inverse", min_sep_m=5.0)
    a1, a2 = baselines(nant)
    uvw = uvw_tracks(enu, a1, a2, hour_angles(ntime, 8.0), MWA_LATITUDE)
    freq = 140.5e6 + 4e6 * np.arange(nchan)
    du = cell_size(uvw, freq, n)
    sky = sky_powerlaw_box(nsrc, rng, 0.3 / du, 0.5, 10.0)
    vis = predict_numpy(uvw, freq, sky, npol=1, noise=0.0, rng=rng)
    gains = random_gains(nant, rng)
    wl = Workload("differentiable", seed, n, n, du, du, uvw, freq, 1, W, O, np.tile(a1, ntime),
                  np.tile(a2, ntime), nant, vis=vis, sky=sky, gains=gains)
    wl.meta.update(nbl=len(a1), ntime=ntime, enu=enu)
    return wl


def subset_antennas(wl, keep_ants):
    """Restrict a workload to baselines between the given antennas (renumbered 0..k-1)."""
    keep_ants = np.asarray(keep_ants)
    remap = -np.ones(wl.nant, dtype=np.int64)
    remap[keep_ants] = np.arange(len(keep_ants))
    rows = np.nonzero((remap[wl.ant1] >= 0) & (remap[wl.ant2] >= 0))[0]
    g = (rows[:, None] * wl.nchan + np.arange(wl.nchan)[None, :]).reshape(-1)
    out = Workload(wl.name + "_subset", wl.seed, wl.nx, wl.ny, wl.du, wl.dv, wl.uvw[rows].copy(),
                   wl.freq.copy(), wl.npol, wl.W, wl.O,
                   remap[wl.ant1[rows]].astype(np.int32), remap[wl.ant2[rows]].astype(np.int32),
                   len(keep_ants), sky=wl.sky)
    if wl.vis is not None:
        out.vis = wl.vis[g].copy()
    if wl.gains is not None:
        out.gains = wl.gains[keep_ants].copy()
    if wl.flags is not None:
        out.flags = wl.flags[g].copy()
    if wl.weights is not None:
        out.weights = wl.weights[g].copy()
    return out


# ---------------------------------------------------------------------------------------------
# Kernel stacks: A-term (per antenna-pair group) combined with a w-plane term
# ---------------------------------------------------------------------------------------------
def _window(eta):
    eta = np.clip(eta, -1.0, 1.0)
    return (1.0 - eta * eta) ** 2


def kernel_stacks(O=4, n_agroups=4, a_support=15, n_wplanes=32, wmax=200.0, seed=3001):
    """512 complex kernels (16 A-terms x 32 w-planes), each [O][O][S][S] with S = 15 + S_w - 1,
    S_w = 7 + 2 round(12 |w_p| / 200) over signed w-plane centres in [-200, 200] lambda.

    The taps are synthetic: a smooth window over the support times an A-term phase screen
    and a w-dependent chirp, normalised so that the taps of each phase slice have unit total
    magnitude. Returns (stack complex64 [total], offset int64 [nk], support int32 [nk],
    wcentres float64 [n_wplanes]).
    """
    rng = np.random.default_rng(seed)
    na = n_agroups * n_agroups
    step = 2.0 * wmax / n_wplanes
    wc = -wmax + step * (np.arange(n_wplanes) + 0.5)
    sw = 7 + 2 * np.rint(12.0 * np.abs(wc) / wmax).astype(np.int64)
    a_phase = rng.uniform(-math.pi, math.pi, (na, 3))
    supports, chunks, offsets = [], [], []
    off = 0
    for a in range(na):
        for p in range(n_wplanes):
            S = int(a_support + sw[p] - 1)
            h = (S - 1) // 2
            ph = np.arange(O) - O // 2
            taps = np.arange(-h, h + 1, dtype=np.float64)
            dy = taps[None, :] - ph[:, None] / O      # [O, S]  (phase row, tap)
            dx = dy
            ry = dy[:, None, :, None]
            rx = dx[None, :, None, :]
            win = _window(ry / (h + 0.5)) * _window(rx / (h + 0.5))
            chirp = math.pi * (wc[p] / wmax) * (rx * rx + ry * ry) / (h + 0.5) ** 2
            screen = a_phase[a, 0] + a_phase[a, 1] * rx / (h + 0.5) + a_phase[a, 2] * ry / (h + 0.5)
            k = win * np.exp(1j * (chirp + 0.3 * screen))
            k /= np.abs(k).sum(axis=(2, 3), keepdims=True)
            chunks.append(k.astype(np.complex64).reshape(-1))
            supports.append(S)
            offsets.append(off)
            off += O * O * S * S
    return (np.concatenate(chunks), np.array(offsets, dtype=np.int64),
            np.array(supports, dtype=np.int32), wc)


def beam_w_stacks(seed=3001, nant=128, nchan=8, ntime=16, n=4096, O=4, nsrc=20, wmax=200.0,
                  n_agroups=4, n_wplanes=32, npol=1):
    """128 antennas, 8 channels, 16 times, 1 polarisation; each visibility selects the kernel
    (A-group pair, w-plane) with A-group = antenna index mod n_agroups and the w-plane holding
    its w;
    4096^2 grid, oversampling 4. The phase centre is tilted from the zenith so that the
    largest |w| over the observation is ``wmax`` wavelengths."""
    rng = np.random.default_rng(seed)
    enu = antenna_layout(nant, 1500.0, rng, "r_inverse", min_sep_m=5.0)
    a1, a2 = baselines(nant)
    freq = 140.5e6 + 4e6 * np.arange(nchan)
    has = hour_angles(ntime, 8.0)
    lo, hi = 0.0, 0.5
    for _ in range(60):  # bisect the zenith offset so that max |w| = wmax
        mid = 0.5 * (lo + hi)
        uvw = uvw_tracks(enu, a1, a2, has, MWA_LATITUDE + mid)
        wm = np.max(np.abs(uvw[:, 2])) * np.max(freq) / C_LIGHT
        if wm > wmax:
            hi = mid
        else:
            lo = mid
    uvw = uvw_tracks(enu, a1, a2, has, MWA_LATITUDE + lo)
    stack, koff, ksup, wc = kernel_stacks(O=O, n_agroups=n_agroups, n_wplanes=n_wplanes,
                                          wmax=wmax, seed=seed)
    n_wplanes = len(wc)
    step = 2.0 * wmax / n_wplanes
    ant1, ant2 = np.tile(a1, ntime), np.tile(a2, ntime)
    wl_lambda = uvw[:, 2][:, None] * freq[None, :] / C_LIGHT  # [nrow, nchan]
    wp = np.clip(np.floor((wl_lambda + wmax) / step), 0, n_wplanes - 1).astype(np.int64)
    agrp = (n_agroups * (ant1 % n_agroups) + (ant2 % n_agroups)).astype(np.int64)
    kidx = (agrp[:, None] * n_wplanes + wp).reshape(-1).astype(np.int32)
    # Cell size: leave room for the largest half support (22 cells) beyond the 80% rule.
    du = cell_size(uvw, freq, n)
    sky = sky_powerlaw_box(nsrc, rng, 0.3 / du, 0.5, 10.0)
    vis = predict_numpy(uvw, freq, sky, npol=npol, noise=0.1, rng=rng)
    wl = Workload("beam_w_stacks", seed, n, n, du, du, uvw, freq, npol, 0, O, ant1, ant2, nant,
                  vis=vis, sky=sky, kernel_stack=stack, kernel_offset=koff,
                  kernel_support=ksup, kernel_index=kidx)
    wl.meta.update(nbl=len(a1), ntime=ntime, wcentres=wc)
    return wl


# ---------------------------------------------------------------------------------------------
# Batched uneven jobs
# ---------------------------------------------------------------------------------------------
def batched_jobs(seed=4001, njobs=96, nmin=1e4, nmax=2e6, fmin=0.05, fmax=0.30,
                 sizes=(512, 1024, 2048, 4096), W=7, O=8, nant=512, nchan=32, ntime=8,
                 make_vis=True, device=None, scale=1.0):
    """``njobs`` independent single-polarisation jobs. Job j keeps N ~ logU[nmin, nmax]
    visibilities after Bernoulli(f) flagging with f ~ U[fmin, fmax]: it draws N/(1-f) random
    (baseline, time, channel) samples of the MWA-scale array, grids them on an n^2 grid with n
    drawn from ``sizes`` and its own 80% cell size. Each sample is one row with its uvw scaled
    to a common reference frequency (so nchan = 1 per job). ``scale`` shrinks N for tests."""
    rng = np.random.default_rng(seed)
    enu = antenna_layout(nant, 1500.0, rng, "r_inverse", min_sep_m=5.0)
    a1, a2 = baselines(nant)
    nbl = len(a1)
    uvw_all = uvw_tracks(enu, a1, a2, hour_angles(ntime, 8.0), MWA_LATITUDE)
    freq_all = 140.5e6 + 1e6 * np.arange(nchan)
    fref = 150e6
    sky = sky_powerlaw_box(50, rng, 0.15, 0.1, 10.0)
    jobs = []
    for j in range(njobs):
        jr = np.random.default_rng(seed * 1000 + j)
        nkeep = int(math.exp(jr.uniform(math.log(nmin), math.log(nmax))) * scale)
        nkeep = max(nkeep, 16)
        f = jr.uniform(fmin, fmax)
        raw = int(round(nkeep / (1.0 - f)))
        row = jr.integers(0, nbl * ntime, raw)
        ch = jr.integers(0, nchan, raw)
        uvw = uvw_all[row] * (freq_all[ch] / fref)[:, None]
        flags = (jr.random(raw) < f).astype(np.uint8)
        n = int(jr.choice(sizes))
        freq = np.array([fref])
        du = cell_size(uvw, freq, n)
        wl = Workload(f"job{j}", seed * 1000 + j, n, n, du, du, uvw, freq, 1, W, O,
                      a1[row % nbl].astype(np.int32), a2[row % nbl].astype(np.int32), nant,
                      flags=flags, sky=sky, noise=0.1)
        if make_vis:
            if device is None:
                wl.vis = predict_numpy(uvw, freq, sky, npol=1, noise=0.1, rng=jr)
            else:
                wl.vis = predict_torch(uvw, freq, sky, 1, 0.1, seed * 1000 + j, device)
        jobs.append(wl)
    return jobs


# ---------------------------------------------------------------------------------------------
# Instrument response for the Stokes conversion: a per-pixel 2 x 2 complex Jones matrix that
# depends on the pixel's direction and on time (hour angle). Synthetic: a smooth dipole-like
# amplitude pattern per feed, a feed-rotation angle that drifts with hour angle and across
# the field, small direction-dependent leakage, and a phase screen. Inputs only.
# ---------------------------------------------------------------------------------------------
def jones_field(nx, ny, hour_angle=0.0, seed=6001, fov_frac=1.0, dtype=np.complex64):
    """complex [ny, nx, 2, 2] Jones matrices J(l, m, t), row-major (J00, J01, J10, J11), with
    l, m the pixel's offsets from the field centre in units of the half field of view."""
    rng = np.random.default_rng(seed)
    l = (np.arange(nx) - nx // 2) / (nx / 2) * fov_frac
    m = (np.arange(ny) - ny // 2) / (ny / 2) * fov_frac
    L, M = np.meshgrid(l, m)
    r2 = L * L + M * M
    # feed amplitudes (never below ~0.35 on the field, so J stays well conditioned)
    ax = 1.0 - 0.45 * (L * L * 0.9 + M * M * 1.1) / 2.0
    ay = 1.0 - 0.45 * (L * L * 1.1 + M * M * 0.9) / 2.0
    c = rng.uniform(-1.0, 1.0, 6)
    phx = 0.4 * c[0] * L + 0.3 * c[1] * M + 0.1 * hour_angle
    phy = 0.3 * c[2] * L + 0.4 * c[3] * M - 0.1 * hour_angle
    chi = 0.5 * hour_angle + 0.15 * c[4] * L - 0.1 * c[5] * M   # feed rotation
    dxy = 0.04 * (L + 0.5j * M) * (1.0 + 0.2 * r2)
    dyx = -0.03 * (M - 0.7j * L)
    gx = ax * np.exp(1j * phx)
    gy = ay * np.exp(1j * phy)
    cs, sn = np.cos(chi), np.sin(chi)
    J = np.empty((ny, nx, 2, 2), dtype=np.complex128)
    # [[gx, gx dxy], [gy dyx, gy]] @ [[cos chi, sin chi], [-sin chi, cos chi]]
    J[..., 0, 0] = gx * (cs - dxy * sn)
    J[..., 0, 1] = gx * (sn + dxy * cs)
    J[..., 1, 0] = gy * (dyx * cs - sn)
    J[..., 1, 1] = gy * (dyx * sn + cs)
    return J.astype(dtype)
