"""Host-only checks of the C ABI: the library loads, exports every function declared in
include/mwagrid.h, the ctypes structures match the C layout (offsets from gcc), and invalid
arguments are rejected with a status and a message before any GPU work.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mwagrid.h")


@pytest.fixture(scope="module")
def mw():
    from paper_0902_0915_amd import mwagrid
    return mwagrid


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mw_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(mw):
    names = _declared_functions()
    assert "mw_grid_plan" in names and "mw_image" in names
    for n in names:
        assert hasattr(mw.lib(), n), n
    out = subprocess.run(["nm", "-D", "--defined-only", mw._LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (mw_[a-z_]+)", out))
    assert set(names) <= exported


def test_struct_layout_matches_c(mw, tmp_path):
    fields = {"mw_instance": mw.MwInstance, "mw_tuning": mw.MwTuning,
              "mw_plan_stats": mw.MwPlanStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mwagrid.h"', 'int main(void){']
    for cname, cls in fields.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f, _ in cls._fields_:
            c_field = {"uvw_m": "uvw_m"}.get(f, f)
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {c_field}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        c, f, v = line.split()
        got[(c, f)] = int(v)
    for cname, cls in fields.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for f, _ in cls._fields_:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)


def test_abi_version(mw):
    assert mw.abi_version() == 5


def _instance(mw, **over):
    uvw = np.zeros((4, 3))
    freq = np.array([150e6])
    d = mw.MwInstance()
    d.nx = d.ny = 64
    d.du = d.dv = 1.0
    d.nrow, d.nchan, d.npol = 4, 1, 1
    d.uvw_m, d.freq_hz = uvw.ctypes.data, freq.ctypes.data
    d.support, d.oversample, d.mem = 7, 8, mw.MW_MEM_HOST
    for k, v in over.items():
        setattr(d, k, v)
    return d, (uvw, freq)


@pytest.mark.parametrize("over,code,needle", [
    (dict(nx=63), 1, "even"),
    (dict(ny=4), 1, "even"),
    (dict(nx=8192), 2, "4096"),
    (dict(du=0.0), 1, "du"),
    (dict(du=float("nan")), 1, "du"),
    (dict(nchan=0), 1, "nchan"),
    (dict(npol=3), 1, "npol"),
    (dict(mem=7), 1, "mem"),
    (dict(support=8), 1, "support"),
    (dict(support=17), 1, "support"),
    (dict(oversample=0), 1, "oversample"),
    (dict(oversample=17), 1, "oversample"),
    (dict(uvw_m=None), 1, "uvw_m"),
    (dict(nrow=1 << 30, nchan=4), 2, "2^31"),
])
def test_plan_rejects_invalid_instances(mw, over, code, needle):
    d, keep = _instance(mw, **over)
    arr = (mw.MwInstance * 1)(d)
    h = ctypes.c_void_p()
    st = mw.lib().mw_grid_plan(ctypes.byref(h), arr, 1, None, None)
    assert st == code
    assert needle in mw.lib().mw_last_error().decode()
    assert h.value is None


def test_plan_rejects_ant_mismatch_and_bad_tuning(mw):
    a1 = np.zeros(4, dtype=np.int32)
    d, keep = _instance(mw, ant1=a1.ctypes.data)
    h = ctypes.c_void_p()
    assert mw.lib().mw_grid_plan(ctypes.byref(h), (mw.MwInstance * 1)(d), 1, None, None) == 1
    d, keep = _instance(mw)
    for bad in (dict(tile=48), dict(split=10), dict(wg_waves=3), dict(order=4), dict(variant=9),
                dict(flush=5), dict(schedule=4)):
        t = mw.MwTuning(**bad)
        st = mw.lib().mw_grid_plan(ctypes.byref(h), (mw.MwInstance * 1)(d), 1, ctypes.byref(t), None)
        assert st == 1, bad
        assert "tuning" in mw.lib().mw_last_error().decode()


def test_calls_on_missing_or_dead_plans(mw):
    lib = mw.lib()
    assert lib.mw_grid_plan(None, None, 1, None, None) == 1
    h = ctypes.c_void_p()
    assert lib.mw_grid_plan(ctypes.byref(h), None, 1, None, None) == 1
    assert lib.mw_grid(None, None, None, None, 0, None) == 1
    assert lib.mw_degrid(None, None, None, None, None, None, None) == 1
    assert lib.mw_image(None, None, None, 1, 1, None) == 1
    assert lib.mw_stokes(None, None, None, None, None) == 1
    bogus = ctypes.c_void_p(0x1000)
    assert lib.mw_stokes(bogus, None, None, None, None) == 5
    assert lib.mw_grid(bogus, None, None, None, 0, None) == 5
    assert b"not live" in lib.mw_last_error()
    assert lib.mw_plan_destroy(bogus) == 5
    assert lib.mw_plan_destroy(None) == 0
    st = mw.MwPlanStats()
    assert lib.mw_plan_info(bogus, 0, ctypes.byref(st)) == 5


def test_last_error_is_per_thread(mw):
    import threading
    lib = mw.lib()
    lib.mw_grid(None, None, None, None, 0, None)
    msgs = {}

    def other():
        msgs["other"] = lib.mw_last_error().decode()

    t = threading.Thread(target=other)
    t.start()
    t.join()
    assert msgs["other"] == ""
    assert lib.mw_last_error().decode() == "plan is NULL"
