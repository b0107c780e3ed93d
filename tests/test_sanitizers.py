"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code (no GPU needed):
the oracle's C loops (gcc), the library's host code (hipcc; the sanitizers on the host pass
only, each after -Xarch_host) with the prolate tables, the autotuner's cache parser on crafted
files, and every C ABI entry point's argument checking. Each driver exits non-zero on a wrong
result, and the sanitizers abort on any memory or undefined-behaviour error."""
import concurrent.futures as cf
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0902_0915_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]
SOURCES = ["abi.cpp", "pswf.cpp", "plan.hip", "grid.hip", "degrid.hip", "image.hip", "fft.hip", "stack.hip",
           "batched.hip", "tuner.cpp", "stokes.hip", "owner.hip", "calib.hip", "weighting.hip", "wstack.hip", "workers.cpp", "runs.hip"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd[:3], r.stdout[-2000:], r.stderr[-4000:])
    return r


def _env(leaks):
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = f"detect_leaks={1 if leaks else 0}:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    return env


def test_oracle_loops_under_sanitizers(tmp_path):
    exe = tmp_path / "orc"
    _run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "oracle.c"),
          os.path.join(SAN, "oracle_driver.c"), "-lm", "-o", str(exe)])
    r = _run([str(exe)], env=_env(True), timeout=120)
    assert "oracle checks passed" in r.stdout


def test_kernel_tables_and_tuner_cache_under_sanitizers(tmp_path):
    exe = tmp_path / "host"
    _run([HIPCC, "-x", "hip", "--offload-host-only", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
          *HOST_SAN, "-I", os.path.join(ROOT, "include"), "-I", CSRC, os.path.join(CSRC, "pswf.cpp"),
          os.path.join(SAN, "host_driver.cpp"), "-o", str(exe)])
    r = _run([str(exe), str(tmp_path)], env=_env(True), timeout=120)
    assert "host checks passed" in r.stdout


def test_abi_argument_checks_under_sanitizers(tmp_path):
    flags = ["-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer", *HOST_SAN,
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        _run([HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(min(8, len(os.sched_getaffinity(0)))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    exe = tmp_path / "abi"
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer", *HOST_SAN[:4], "-x", "c",
          os.path.join(SAN, "abi_driver.c"), "-x", "none", *objs, "-I", os.path.join(ROOT, "include"),
          "-L/opt/rocm/lib", "-lrocfft", "-Wl,-rpath,/opt/rocm/lib", "-o", str(exe)])
    # leak checking off: the HIP runtime's own start-up allocations outlive main
    r = _run([str(exe)], env=_env(False), timeout=120)
    assert "abi checks passed" in r.stdout
