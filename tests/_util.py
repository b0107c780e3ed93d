"""Shared helpers for the GPU parity tests (not collected as tests)."""
import numpy as np

import oracle as orc


def nl2(got, ref):
    """Normalised L2 error ||got - ref|| / ||ref||."""
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    den = np.linalg.norm(ref.ravel())
    return float(np.linalg.norm((got - ref).ravel()) / (den if den > 0 else 1.0))


def oracle_positions(wl, weights=None):
    return orc.positions(wl.uvw, wl.freq, wl.nx, wl.ny, wl.du, wl.dv, wl.W, wl.O,
                         flags=wl.flags, weights=weights)


def oracle_grid(wl, vis, weights=None, gains=None):
    pos, keep, _ = oracle_positions(wl, weights)
    return orc.grid(pos, keep, vis, wl.nx, wl.ny, wl.W, wl.O, nchan=wl.nchan, weights=weights,
                    gains=gains, ant1=wl.ant1 if gains is not None else None,
                    ant2=wl.ant2 if gains is not None else None)


def to_dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def to_host(t):
    return t.detach().cpu().numpy()


def coverage(pos, keep, nx, ny, W):
    """Number of kept groups whose W x W footprint covers each cell, int64 [ny, nx]."""
    kp = np.asarray(pos)[np.asarray(keep, dtype=bool)]
    h = (W - 1) // 2
    c = np.bincount(kp[:, 1].astype(np.int64) * nx + kp[:, 0], minlength=nx * ny)
    c = c.reshape(ny, nx).astype(np.int64)
    # box sum of width W along each axis (footprints never leave the grid)
    p = np.zeros((ny + W, nx), np.int64)
    p[h + 1:h + 1 + ny] = np.cumsum(c, axis=0)
    p[h + 1 + ny:] = p[h + ny]
    c = p[W:W + ny] - p[0:ny]
    q = np.zeros((ny, nx + W), np.int64)
    q[:, h + 1:h + 1 + nx] = np.cumsum(c, axis=1)
    q[:, h + 1 + nx:] = q[:, h + nx][:, None]
    return q[:, W:W + nx] - q[:, 0:nx]


def region_errors(got, ref, cover, dense_frac=0.01):
    """Normalised L2 error of a grid [npol, ny, nx] over three regions of cells: the densest
    dense_frac of the covered cells (by footprint count), the rest of the covered cells, and
    the cells no footprint covers (returned as the number of nonzero values there in got and
    in ref, which must both be 0)."""
    covered = cover > 0
    vals = cover[covered]
    thr = np.quantile(vals, 1.0 - dense_frac) if vals.size else 0
    dense = covered & (cover >= thr)
    rest = covered & ~dense
    out = {}
    for name, m in (("dense", dense), ("rest", rest)):
        out[name] = nl2(np.asarray(got)[:, m], np.asarray(ref)[:, m]) if m.any() else 0.0
    zero = ~covered
    out["zero_nonzero_got"] = int(np.count_nonzero(np.asarray(got)[:, zero]))
    out["zero_nonzero_ref"] = int(np.count_nonzero(np.asarray(ref)[:, zero]))
    out["cells"] = (int(dense.sum()), int(rest.sum()), int(zero.sum()))
    return out
