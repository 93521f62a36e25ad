"""Host-side checks of bench.py that need no GPU: the one-GPU contract and the
traffic figure's tie to the profiled kernel sources."""
import hashlib
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_only_while_sources_match():
    """The committed HBM traffic is reported only for the kernel sources it was measured on."""
    b = load_bench()
    meta = json.load(open(os.path.join(ROOT, "profiles", "forward_kernel_covering_1M_p3_c2.json")))
    h = hashlib.sha256()
    for f in meta["source_files"]:
        h.update(open(os.path.join(ROOT, "paper_2507_21686_amd", "csrc", f), "rb").read())
    match = h.hexdigest()[:16] == meta["source_sha256_16"]
    got = b.measured_traffic()
    assert got == (meta["traffic_bytes_per_launch"] if match else None)
    scaled = (meta["fetch_kib"] * meta["fetch_scale"] + meta["write_kib"] * meta["write_scale"]) * 1024
    assert abs(scaled - meta["traffic_bytes_per_launch"]) <= 1024
