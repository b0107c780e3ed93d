"""Thin ctypes binding of libmwagrid (include/mwagrid.h): argument marshalling only.

Every step of the computation runs in the library's HIP kernels; torch provides device
memory and streams. Importing this module loads ``libmwagrid.so`` from the package
directory and raises ``RuntimeError`` if it has not been built (``python -m
paper_0902_0915_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

# torch first: the library then binds to the HIP runtime torch has already loaded, so both
# see the same devices, contexts and allocations.
import torch  # noqa: E402,F401

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmwagrid.so")
if not os.path.exists(_LIB_PATH):
    raise RuntimeError(f"libmwagrid.so is not built ({_LIB_PATH}); run "
                       "`python -m paper_0902_0915_amd.build` (hipcc, gfx950)")
_lib = ctypes.CDLL(_LIB_PATH)

MW_OK, MW_ERR_INVALID_ARG, MW_ERR_UNSUPPORTED, MW_ERR_ALLOC, MW_ERR_HIP, MW_ERR_STATE = range(6)
MW_MEM_HOST, MW_MEM_DEVICE = 0, 1
STATUS_NAMES = {0: "MW_OK", 1: "MW_ERR_INVALID_ARG", 2: "MW_ERR_UNSUPPORTED",
                3: "MW_ERR_ALLOC", 4: "MW_ERR_HIP", 5: "MW_ERR_STATE"}

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


class MwInstance(ctypes.Structure):
    _fields_ = [("nx", _i32), ("ny", _i32), ("du", ctypes.c_double), ("dv", ctypes.c_double),
                ("nrow", _i64), ("nchan", _i32), ("npol", _i32),
                ("uvw_m", _vp), ("freq_hz", _vp), ("flags", _vp), ("weights", _vp),
                ("ant1", _vp), ("ant2", _vp), ("nant", _i32),
                ("support", _i32), ("oversample", _i32),
                ("kernel_stack", _vp), ("kernel_offset", _vp), ("kernel_support", _vp),
                ("nkernel", _i32), ("kernel_elems", _i64), ("kernel_index", _vp),
                ("mem", _i32), ("weighting", _i32), ("robust", ctypes.c_float),
                ("wlo", ctypes.c_double), ("whi", ctypes.c_double)]


class MwTuning(ctypes.Structure):
    _fields_ = [("tile", _i32), ("split", _i32), ("wg_waves", _i32), ("order", _i32),
                ("variant", _i32), ("flush", _i32), ("autotune", _i32), ("schedule", _i32)]


class MwPlanStats(ctypes.Structure):
    _fields_ = [("ngroups", _i64), ("nkept", _i64), ("nflagged", _i64), ("noutside", _i64),
                ("ntiles", _i32), ("nwork", _i32), ("tile", _i32), ("split", _i32),
                ("wg_waves", _i32), ("order", _i32), ("variant", _i32), ("flush", _i32),
                ("schedule", _i32), ("plan_bytes", _i64), ("batched", _i32), ("pad0", _i32)]


_PP = ctypes.POINTER(ctypes.c_void_p)
_lib.mw_grid_plan.argtypes = [ctypes.POINTER(_vp), ctypes.POINTER(MwInstance), _i32,
                              ctypes.POINTER(MwTuning), _vp]
_lib.mw_grid.argtypes = [_vp, _PP, _PP, _PP, _i32, _vp]
_lib.mw_grid_noalloc.argtypes = [_vp, _PP, _PP, _PP, _i32, _vp]
_lib.mw_degrid.argtypes = [_vp, _PP, _PP, _PP, _PP, _PP, _vp]
_lib.mw_image.argtypes = [_vp, _PP, _PP, _i32, _i32, _vp]
_lib.mw_stokes.argtypes = [_vp, _PP, _PP, _PP, _vp]
_lib.mw_predict.argtypes = [_vp, _i32, _vp, _i32, _vp, _vp, _i32, _vp]
_lib.mw_solve_gains.argtypes = [_vp, _i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp]
_lib.mw_peel.argtypes = [_vp, _i32, _vp, _vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp]
_lib.mw_wstack_combine.argtypes = [_vp, _PP, _vp, _i32, _vp]
_lib.mw_plan_info.argtypes = [_vp, _i32, ctypes.POINTER(MwPlanStats)]
_lib.mw_plan_positions.argtypes = [_vp, _i32, _vp]
_lib.mw_plan_order.argtypes = [_vp, _i32, _vp]
_lib.mw_plan_tables.argtypes = [_vp, _i32, _vp, _vp, _vp]
_lib.mw_plan_destroy.argtypes = [_vp]
_lib.mw_plan_set_timing.argtypes = [_vp, _i32]
_lib.mw_plan_kernel_ms.argtypes = [_vp, _i32, ctypes.POINTER(ctypes.c_float),
                                   ctypes.POINTER(ctypes.c_float)]
_lib.mw_last_error.argtypes = []
_lib.mw_last_error.restype = ctypes.c_char_p
_lib.mw_abi_version.argtypes = []
_lib.mw_abi_version.restype = _i32
for _f in ("mw_grid_plan", "mw_grid", "mw_degrid", "mw_image", "mw_plan_info",
           "mw_plan_positions", "mw_plan_order", "mw_plan_tables", "mw_plan_destroy", "mw_plan_set_timing",
           "mw_plan_kernel_ms", "mw_stokes", "mw_grid_noalloc", "mw_predict", "mw_solve_gains",
           "mw_peel", "mw_wstack_combine"):
    getattr(_lib, _f).restype = _i32


class MwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _check(status):
    if status != MW_OK:
        raise MwError(status, _lib.mw_last_error().decode(errors="replace"))


def lib():
    return _lib


def abi_version():
    return int(_lib.mw_abi_version())


def _ptr_array(ptrs):
    arr = (ctypes.c_void_p * len(ptrs))(*[p if p else None for p in ptrs])
    return ctypes.cast(arr, _PP), arr


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_ptr(t, dtype=None, what="tensor"):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what} must be {dtype}, got {t.dtype}")
    return t.data_ptr()


@dataclass
class InstanceSpec:
    """One gridding instance (host numpy arrays or device torch tensors, not mixed)."""
    nx: int
    ny: int
    du: float
    dv: float
    uvw: object              # [nrow, 3] float64 metres
    freq: object             # [nchan] float64 Hz
    npol: int = 1
    W: int = 7
    O: int = 8
    flags: object = None     # [ngroups] uint8
    weights: object = None   # [ngroups] float32
    ant1: object = None      # [nrow] int32
    ant2: object = None
    nant: int = 0
    kernel_stack: object = None    # complex64 ragged
    kernel_offset: object = None   # int64 [nkernel]
    kernel_support: object = None  # int32 [nkernel]
    kernel_index: object = None    # int32 [ngroups]
    weighting: str = "natural"     # "natural", "uniform" or "robust"
    robust: float = 0.0            # Briggs robustness for "robust"
    wrange: tuple = (0.0, 0.0)     # (wlo, whi): grid only wlo <= w < whi (one w-plane)

    @classmethod
    def from_workload(cls, wl, with_ants=True, with_weights=True):
        return cls(wl.nx, wl.ny, wl.du, wl.dv, wl.uvw, wl.freq, wl.npol, wl.W, wl.O,
                   flags=wl.flags, weights=wl.weights if with_weights else None,
                   ant1=wl.ant1 if with_ants else None, ant2=wl.ant2 if with_ants else None,
                   nant=wl.nant if with_ants else 0, kernel_stack=wl.kernel_stack,
                   kernel_offset=wl.kernel_offset, kernel_support=wl.kernel_support,
                   kernel_index=wl.kernel_index)


def _host_arrays(spec):
    """Contiguous host copies with the ABI dtypes; returns (dict of arrays, keepalive)."""
    conv = {
        "uvw": (spec.uvw, np.float64), "freq": (spec.freq, np.float64),
        "flags": (spec.flags, np.uint8), "weights": (spec.weights, np.float32),
        "ant1": (spec.ant1, np.int32), "ant2": (spec.ant2, np.int32),
        "kernel_stack": (spec.kernel_stack, np.complex64),
        "kernel_offset": (spec.kernel_offset, np.int64),
        "kernel_support": (spec.kernel_support, np.int32),
        "kernel_index": (spec.kernel_index, np.int32),
    }
    out = {}
    for k, (a, dt) in conv.items():
        out[k] = None if a is None else np.ascontiguousarray(np.asarray(a), dtype=dt)
    return out


def _instance_struct(spec):
    a = _host_arrays(spec)

    def p(x):
        return None if x is None else x.ctypes.data

    nrow = a["uvw"].shape[0]
    d = MwInstance()
    d.nx, d.ny, d.du, d.dv = int(spec.nx), int(spec.ny), float(spec.du), float(spec.dv)
    d.nrow, d.nchan, d.npol = nrow, a["freq"].shape[0], int(spec.npol)
    d.uvw_m, d.freq_hz, d.flags, d.weights = p(a["uvw"]), p(a["freq"]), p(a["flags"]), p(a["weights"])
    d.ant1, d.ant2, d.nant = p(a["ant1"]), p(a["ant2"]), int(spec.nant)
    d.support = int(spec.W) if a["kernel_stack"] is None else 0
    d.oversample = int(spec.O)
    if a["kernel_stack"] is not None:
        d.kernel_stack, d.kernel_offset = p(a["kernel_stack"]), p(a["kernel_offset"])
        d.kernel_support, d.nkernel = p(a["kernel_support"]), a["kernel_support"].shape[0]
        d.kernel_elems, d.kernel_index = a["kernel_stack"].shape[0], p(a["kernel_index"])
    d.mem = MW_MEM_HOST
    d.weighting = {"natural": 0, "uniform": 1, "robust": 2}[spec.weighting]
    d.robust = float(spec.robust)
    d.wlo, d.whi = float(spec.wrange[0]), float(spec.wrange[1])
    return d, a


class Plan:
    """A gridding plan over one or more instances (mw_grid_plan)."""

    def __init__(self, specs, tuning=None, stream=None):
        import torch
        if isinstance(specs, InstanceSpec):
            specs = [specs]
        self.specs = list(specs)
        structs, keep = [], []
        for sp in self.specs:
            d, a = _instance_struct(sp)
            structs.append(d)
            keep.append(a)
        arr = (MwInstance * len(structs))(*structs)
        tun = None
        if tuning is not None:
            tun = MwTuning(**{k: int(v) for k, v in tuning.items()})
        handle = ctypes.c_void_p()
        torch.cuda.init()
        _check(_lib.mw_grid_plan(ctypes.byref(handle), arr, len(structs),
                                 ctypes.byref(tun) if tun is not None else None,
                                 _stream_handle(stream)))
        self._h = handle
        self.device = torch.device("cuda", torch.cuda.current_device())

    # ---- lifecycle ---------------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(_lib.mw_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        if self._h is None:
            raise MwError(MW_ERR_STATE, "plan is closed")
        return self._h

    @property
    def ninst(self):
        return len(self.specs)

    # ---- queries -----------------------------------------------------------------------
    def info(self, inst=-1):
        st = MwPlanStats()
        _check(_lib.mw_plan_info(self.handle, inst, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in MwPlanStats._fields_}

    def positions(self, inst=0):
        sp = self.specs[inst]
        ng = np.asarray(sp.uvw).shape[0] * np.asarray(sp.freq).shape[0]
        out = np.empty((ng, 4), dtype=np.int32)
        _check(_lib.mw_plan_positions(self.handle, inst, out.ctypes.data))
        return out

    def order(self, inst=0):
        """mw_plan_order: the input index of each kept group in the gridding order."""
        out = np.empty(self.info(inst)["nkept"], dtype=np.uint32)
        _check(_lib.mw_plan_order(self.handle, inst, out.ctypes.data))
        return out

    def tables(self, inst=0):
        sp = self.specs[inst]
        tab = np.empty((sp.O, sp.W), dtype=np.float32)
        cx = np.empty(sp.nx, dtype=np.float32)
        cy = np.empty(sp.ny, dtype=np.float32)
        _check(_lib.mw_plan_tables(self.handle, inst, tab.ctypes.data, cx.ctypes.data,
                                   cy.ctypes.data))
        return tab, cx, cy

    def set_timing(self, enable=True):
        _check(_lib.mw_plan_set_timing(self.handle, 1 if enable else 0))

    def kernel_ms(self, inst=0):
        """(gridder ms, merge ms) of the last timed grid call of instance ``inst``."""
        g, m = ctypes.c_float(), ctypes.c_float()
        _check(_lib.mw_plan_kernel_ms(self.handle, inst, ctypes.byref(g), ctypes.byref(m)))
        return g.value, m.value

    # ---- compute -----------------------------------------------------------------------
    def _as_list(self, x):
        if x is None:
            return [None] * self.ninst
        if isinstance(x, (list, tuple)):
            if len(x) != self.ninst:
                raise ValueError("one entry per instance is required")
            return list(x)
        if self.ninst != 1:
            raise ValueError("pass a list with one entry per instance")
        return [x]

    def _ngroups(self, i):
        sp = self.specs[i]
        return np.asarray(sp.uvw).shape[0] * np.asarray(sp.freq).shape[0]

    def _check_shape(self, t, shape, what):
        if t is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"{what} has shape {tuple(t.shape)}, expected {tuple(shape)}")

    def _check_vis(self, lst, what):
        for i, t in enumerate(lst):
            self._check_shape(t, (self._ngroups(i), self.specs[i].npol), what)

    def _check_grid(self, lst, what):
        for i, t in enumerate(lst):
            sp = self.specs[i]
            self._check_shape(t, (sp.npol, sp.ny, sp.nx), what)

    def _check_gains(self, lst):
        for i, t in enumerate(lst):
            if self.specs[i].nant > 0:  # an instance without antennas is refused by the library
                self._check_shape(t, (self.specs[i].nant,), "gains")

    def new_grids(self):
        import torch
        return [torch.empty((sp.npol, sp.ny, sp.nx), dtype=torch.complex64, device=self.device)
                for sp in self.specs]

    def grid(self, vis, gains=None, out=None, accumulate=False, stream=None, noalloc=False):
        """mw_grid; noalloc=True calls mw_grid_noalloc (static scratch, no allocation; out
        should then be given so that the binding allocates nothing either)."""
        import torch
        vis_l, gains_l = self._as_list(vis), self._as_list(gains)
        outs = self._as_list(out) if out is not None else self.new_grids()
        self._check_vis(vis_l, "vis")
        self._check_grid(outs, "grid")
        self._check_gains(gains_l)
        vp, _k1 = _ptr_array([_dev_ptr(v, torch.complex64, "vis") for v in vis_l])
        gp, _k2 = _ptr_array([_dev_ptr(g, torch.complex64, "gains") for g in gains_l])
        op, _k3 = _ptr_array([_dev_ptr(o, torch.complex64, "grid") for o in outs])
        fn = _lib.mw_grid_noalloc if noalloc else _lib.mw_grid
        _check(fn(self.handle, vp, gp if gains is not None else None, op,
                  1 if accumulate else 0, _stream_handle(stream)))
        return outs if isinstance(vis, (list, tuple)) else outs[0]

    def degrid(self, grid, gains=None, vis_in=None, want_grad_gains=False, out=None,
               stream=None):
        import torch
        g_l, gains_l, vin_l = self._as_list(grid), self._as_list(gains), self._as_list(vis_in)
        if out is None:
            outs = []
            for sp in self.specs:
                ng = np.asarray(sp.uvw).shape[0] * np.asarray(sp.freq).shape[0]
                outs.append(torch.empty((ng, sp.npol), dtype=torch.complex64, device=self.device))
        else:
            outs = self._as_list(out)
        gg = [torch.empty(sp.nant, dtype=torch.complex64, device=self.device) if want_grad_gains
              else None for sp in self.specs]
        self._check_grid(g_l, "grid")
        self._check_vis(outs, "vis_out")
        self._check_vis(vin_l, "vis_in")
        self._check_gains(gains_l)
        gp, _k1 = _ptr_array([_dev_ptr(x, torch.complex64, "grid") for x in g_l])
        ga, _k2 = _ptr_array([_dev_ptr(x, torch.complex64, "gains") for x in gains_l])
        vi, _k3 = _ptr_array([_dev_ptr(x, torch.complex64, "vis_in") for x in vin_l])
        vo, _k4 = _ptr_array([_dev_ptr(x, torch.complex64, "vis_out") for x in outs])
        gr, _k5 = _ptr_array([_dev_ptr(x, torch.complex64, "grad_gains") for x in gg])
        _check(_lib.mw_degrid(self.handle, gp, ga if gains is not None else None,
                              vi if vis_in is not None else None, vo,
                              gr if want_grad_gains else None, _stream_handle(stream)))
        single = not isinstance(grid, (list, tuple))
        if want_grad_gains:
            return (outs[0], gg[0]) if single else (outs, gg)
        return outs[0] if single else outs

    def image(self, x, direction=1, correct=True, out=None, stream=None):
        import torch
        x_l = self._as_list(x)
        outs = self._as_list(out) if out is not None else [torch.empty_like(t) for t in x_l]
        self._check_grid(x_l, "in")
        self._check_grid(outs, "out")
        ip, _k1 = _ptr_array([_dev_ptr(t, torch.complex64, "in") for t in x_l])
        op, _k2 = _ptr_array([_dev_ptr(t, torch.complex64, "out") for t in outs])
        _check(_lib.mw_image(self.handle, ip, op, int(direction), 1 if correct else 0,
                             _stream_handle(stream)))
        return outs if isinstance(x, (list, tuple)) else outs[0]


    def stokes(self, images, jones=None, out=None, stream=None):
        """Stokes I, Q, U, V (float32 [4, ny, nx]) of the XX, XY, YX, YY images; jones: None
        (ideal feeds) or complex64 [ny, nx, 2, 2] per instance."""
        import torch
        x_l, j_l = self._as_list(images), self._as_list(jones)
        self._check_grid(x_l, "images")
        outs = (self._as_list(out) if out is not None else
                [torch.empty((4, sp.ny, sp.nx), dtype=torch.float32, device=self.device)
                 for sp in self.specs])
        for i, sp in enumerate(self.specs):
            self._check_shape(j_l[i], (sp.ny, sp.nx, 2, 2), "jones")
            self._check_shape(outs[i], (4, sp.ny, sp.nx), "out")
        ip, _k1 = _ptr_array([_dev_ptr(t, torch.complex64, "images") for t in x_l])
        jp, _k2 = _ptr_array([_dev_ptr(t, torch.complex64, "jones") for t in j_l])
        op, _k3 = _ptr_array([_dev_ptr(t, torch.float32, "out") for t in outs])
        _check(_lib.mw_stokes(self.handle, ip, jp if jones is not None else None, op,
                              _stream_handle(stream)))
        return outs if isinstance(images, (list, tuple)) else outs[0]


    # ---- calibration ----------------------------------------------------------------------
    def predict(self, sources, gains=None, out=None, accumulate=False, inst=0, stream=None):
        """Visibilities of point sources (device float64 [nsrc, 3] of l, m, flux) at the
        instance's uvw and frequencies, times g1 conj(g2) when gains are given."""
        import torch
        sp = self.specs[inst]
        src = torch.as_tensor(sources, dtype=torch.float64).reshape(-1, 3).contiguous().to(self.device)
        if out is None:
            out = torch.empty((self._ngroups(inst), sp.npol), dtype=torch.complex64, device=self.device)
        self._check_shape(out, (self._ngroups(inst), sp.npol), "out")
        if gains is not None:
            self._check_shape(gains, (sp.nant,), "gains")
        _check(_lib.mw_predict(self.handle, inst, _dev_ptr(src, torch.float64, "sources"), src.shape[0],
                               _dev_ptr(gains, torch.complex64, "gains"),
                               _dev_ptr(out, torch.complex64, "out"), 1 if accumulate else 0,
                               _stream_handle(stream)))
        return out

    def solve_gains(self, vis, model, weights=None, gains=None, niter=10, inst=0, stream=None):
        """StEFCal solution of vis ~ g1 conj(g2) model; returns (gains, relative last step)."""
        import torch
        sp = self.specs[inst]
        shape = (self._ngroups(inst), sp.npol)
        self._check_shape(vis, shape, "vis")
        self._check_shape(model, shape, "model")
        g = (torch.ones(sp.nant, dtype=torch.complex64, device=self.device) if gains is None
             else gains.clone())
        rel = torch.zeros(1, dtype=torch.float32, device=self.device)
        if weights is not None:
            self._check_shape(weights, (self._ngroups(inst),), "weights")
        _check(_lib.mw_solve_gains(self.handle, inst, _dev_ptr(vis, torch.complex64, "vis"),
                                   _dev_ptr(model, torch.complex64, "model"),
                                   _dev_ptr(weights, torch.float32, "weights"),
                                   _dev_ptr(g, torch.complex64, "gains"), int(niter),
                                   _dev_ptr(rel, torch.float32, "rel"), _stream_handle(stream)))
        return g, rel

    def peel(self, vis, sources, weights=None, niter=10, inst=0, stream=None):
        """The calibration measurement loop over a catalogue (host float64 [nsrc, 3] of l, m,
        flux): returns (residual, gains [nsrc, nant] in catalogue order, relative last steps)."""
        import torch
        sp = self.specs[inst]
        shape = (self._ngroups(inst), sp.npol)
        self._check_shape(vis, shape, "vis")
        src = np.ascontiguousarray(np.asarray(sources, dtype=np.float64).reshape(-1, 3))
        nsrc = src.shape[0]
        resid = torch.empty(shape, dtype=torch.complex64, device=self.device)
        gains = torch.empty((max(nsrc, 1), sp.nant), dtype=torch.complex64, device=self.device)
        rel = torch.zeros(max(nsrc, 1), dtype=torch.float32, device=self.device)
        if weights is not None:
            self._check_shape(weights, (self._ngroups(inst),), "weights")
        _check(_lib.mw_peel(self.handle, inst, _dev_ptr(vis, torch.complex64, "vis"), src.ctypes.data, nsrc,
                            _dev_ptr(weights, torch.float32, "weights"), int(niter),
                            _dev_ptr(resid, torch.complex64, "resid"),
                            _dev_ptr(gains, torch.complex64, "gains"),
                            _dev_ptr(rel, torch.float32, "rel"), _stream_handle(stream)))
        return resid, gains[:nsrc], rel[:nsrc]


    def wstack_combine(self, images, out=None, accumulate=False, stream=None):
        """Sum of the instances' images (one w-plane each) with their planes' w-term phase."""
        import torch
        x_l = self._as_list(images)
        self._check_grid(x_l, "images")
        sp = self.specs[0]
        if out is None:
            out = torch.empty((sp.npol, sp.ny, sp.nx), dtype=torch.complex64, device=self.device)
        self._check_shape(out, (sp.npol, sp.ny, sp.nx), "out")
        ip, _k1 = _ptr_array([_dev_ptr(t, torch.complex64, "images") for t in x_l])
        _check(_lib.mw_wstack_combine(self.handle, ip, _dev_ptr(out, torch.complex64, "out"),
                                      1 if accumulate else 0, _stream_handle(stream)))
        return out


def wstack_specs(spec, nplanes):
    """One InstanceSpec per w-plane: nplanes equal ranges of w = (w_m f)/c spanning the
    instance's samples (the last range closed just above the largest w)."""
    import dataclasses
    uvw = np.asarray(spec.uvw, dtype=np.float64)
    freq = np.asarray(spec.freq, dtype=np.float64)
    w = uvw[:, 2:3] * freq[None, :] / 299792458.0
    lo, hi = float(w.min()), float(w.max())
    hi = hi + max(1e-9, 1e-12 * abs(hi))
    edges = np.linspace(lo, hi, nplanes + 1)
    return [dataclasses.replace(spec, wrange=(float(edges[k]), float(edges[k + 1]))) for k in range(nplanes)]


def _grid_image_function():
    import torch

    class GridImage(torch.autograd.Function):
        """image = image(grid(g1 conj(g2) V)) with the hand-written adjoints as backward.

        forward(vis [ngroups, npol] complex64, gains [nant] complex64 or None, plan, correct)
        Gradients follow torch's convention for real losses (dL/dRe + i dL/dIm).
        """

        @staticmethod
        def forward(ctx, vis, gains, plan, correct=True):
            vis = vis.contiguous()
            g = gains.contiguous() if gains is not None else None
            grid = plan.grid(vis, gains=g)
            img = plan.image(grid, direction=1, correct=correct)
            ctx.plan, ctx.correct = plan, correct
            ctx.save_for_backward(vis, g if g is not None else torch.empty(0, device=vis.device))
            ctx.has_gains = g is not None
            return img

        @staticmethod
        def backward(ctx, grad_img):
            vis, g = ctx.saved_tensors
            plan = ctx.plan
            grad_grid = plan.image(grad_img.contiguous(), direction=-1, correct=ctx.correct)
            need_g = ctx.has_gains and ctx.needs_input_grad[1]
            if ctx.has_gains:
                res = plan.degrid(grad_grid, gains=g, vis_in=vis if need_g else None,
                                  want_grad_gains=need_g)
                gv, gg = res if need_g else (res, None)
            else:
                gv, gg = plan.degrid(grad_grid), None
            return (gv if ctx.needs_input_grad[0] else None), gg, None, None

    return GridImage


_GridImage = None


def grid_image(vis, gains, plan, correct=True):
    """Differentiable image of (gain-corrupted) visibilities: see ``GridImage``."""
    global _GridImage
    if _GridImage is None:
        _GridImage = _grid_image_function()
    return _GridImage.apply(vis, gains, plan, correct)
