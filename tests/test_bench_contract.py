"""bench.py's command-line contract and the consistency of its measured-traffic record with
the committed profile it cites (no GPU needed)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout + r.stderr
    assert r.stdout.strip() == ""  # no JSON line for a refused run


def test_traffic_record_matches_its_profile():
    b = _bench_module()
    m = b.MEASURED_TRAFFIC
    text = open(os.path.join(ROOT, m["profile"]), encoding="utf-8").read()
    # the profile quotes the same per-dispatch counters (KiB) and the same copy-probe scales
    assert f"{int(round(m['fetch_kib'])):,}" in text
    assert f"{int(round(m['write_kib'])):,}" in text
    assert f"**{m['fetch_scale']}**" in text and f"**{m['write_scale']}**" in text
    # and the bytes it implies are what the profile's table states, to 1 MB
    implied = (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"]) * 1024
    assert f"**{implied / 1e9:.3f} GB**" in text


def test_traffic_is_reported_only_for_the_measured_sources():
    b = _bench_module()
    got = b.gridder_traffic()
    m = b.MEASURED_TRAFFIC
    expected = int((m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"]) * 1024)
    assert got in (None, expected)
    # a different source set never matches the recorded hash
    saved = b.GRIDDER_SOURCES
    try:
        b.GRIDDER_SOURCES = saved[:-1]
        assert b.gridder_traffic() is None
    finally:
        b.GRIDDER_SOURCES = saved
