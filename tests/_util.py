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
