"""Host-side checks of the benchmark's command line (no GPU): several GPUs are
refused with a message, and the committed HBM-traffic record is keyed to the
kernel sources it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_several_gpus_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_traffic_record_is_keyed_to_sources():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    b = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(b)
    h = b.kernel_source_hash()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["k_forward/C1"]
    assert rec["hbm_bytes_per_launch"] > 0 and rec["fetch_scale"] > 0 and rec["write_scale"] > 0
    # a record taken on other sources is not used
    got = b.load_traffic("k_forward/C1")
    assert got == (rec["hbm_bytes_per_launch"] if rec["source_hash"] == h else None)
    assert b.load_traffic("no such kernel") is None
