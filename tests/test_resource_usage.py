"""No kernel of the library spills registers to scratch memory (no GPU needed: the compiler's
resource-usage report of every HIP source, built for gfx950 with the library's flags). A
spill turns a kernel's register traffic into memory traffic and costs it many times over;
this check catches it at build time rather than in a benchmark."""
import concurrent.futures as cf
import os
import re
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0902_0915_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-x", "hip", "-O3", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
         "-Rpass-analysis=kernel-resource-usage"]


def _report(src, outdir):
    obj = os.path.join(outdir, os.path.basename(src) + ".o")
    r = subprocess.run([HIPCC, *FLAGS, "-c", src, "-o", obj], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    kernels, name = {}, None
    for line in r.stderr.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            name = m.group(1)
            kernels[name] = {}
            continue
        m = re.search(r"(ScratchSize \[bytes/lane\]|VGPRs Spill|SGPRs Spill): (\d+)", line)
        if m and name:
            kernels[name][m.group(1)] = int(m.group(2))
    return kernels


def test_no_kernel_spills(tmp_path):
    sources = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    with cf.ThreadPoolExecutor(min(8, len(os.sched_getaffinity(0)))) as ex:
        reports = dict(zip(sources, ex.map(lambda s: _report(s, str(tmp_path)), sources)))
    nkernels = sum(len(k) for k in reports.values())
    assert nkernels > 50, nkernels  # the report was parsed
    bad = [(os.path.basename(s), k, v) for s, ks in reports.items() for k, v in ks.items()
           if any(v.get(f, 0) for f in ("ScratchSize [bytes/lane]", "VGPRs Spill", "SGPRs Spill"))]
    assert not bad, bad
