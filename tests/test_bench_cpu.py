"""bench.py on the host: it refuses more than one GPU before touching any
device, and reports the recorded HBM traffic only for the configuration and
kernel form it was taken for, and only while the kernel sources are the ones
it was taken from."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_traffic_record_matches_sources_and_kernel_form(tmp_path):
    b = _bench()
    with open(b.TRAFFIC_FILE) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for rel in rec["source_files"]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    fused = bool(rec.get("fused"))
    got = b.measured_traffic(rec["config"], fused)
    if h.hexdigest() == rec["source_sha256"]:
        assert got == rec["traffic_bytes_per_launch"]
    else:
        assert got is None
    # another configuration or kernel form never takes the figure
    assert b.measured_traffic(rec["config"] + "/other", fused) is None
    assert b.measured_traffic(rec["config"], not fused) is None
    # a record whose hash no longer matches gives none
    stale = dict(rec, source_sha256="0" * 64)
    p = tmp_path / "traffic.json"
    p.write_text(json.dumps(stale))
    b.TRAFFIC_FILE = str(p)
    assert b.measured_traffic(rec["config"], fused) is None


def test_roofline_is_the_ceiling_that_takes_longer():
    b = _bench()
    # the headline's fused launch: 663 MFLOP of useful work and 308 MB of
    # algorithmic bytes in 114 us; HBM alone needs 38.5 us, FP32 alone 4.2 us
    flops, nbytes, us = 26.0 * 25.5e6, 308e6, 114.0
    bound, other = b.rooflines(flops, us, nbytes)
    assert bound["bound"] == "hbm" and other["bound"] == "alu"
    assert abs(bound["frac"] - nbytes / (us * 1e-6) / 8e12) < 1e-12
    assert abs(other["frac"] - flops / (us * 1e-6) / 157.3e12) < 1e-12
    assert abs(bound["flop_per_byte"] - flops / nbytes) < 1e-12
    # the same work with few bytes is bound by the FP32 ceiling
    bound, other = b.rooflines(flops, us, 1e6)
    assert bound["bound"] == "alu" and other["bound"] == "hbm"
    # no lists (linked cells): only the FP32 ceiling
    bound, other = b.rooflines(flops, us, None)
    assert bound["bound"] == "alu" and other is None
