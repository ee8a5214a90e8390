"""Host-only checks of bench.py: the one-GPU contract and the roofline
arithmetic of its JSON line (no GPU, no torch device calls)."""
import importlib.util
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_mfma_roofline_fraction():
    b = _bench()
    # 2.199e12 int8 ops in 0.66 ms: 3.33 POP/s of the 5.0 peak
    r = b.mfma_roofline(2.0 * 65536 ** 2 * 256, 0.66, "unit")
    assert r["bound"] == "mfma" and r["unit"] == "TOP/s" and r["peak"] == 5000.0
    assert abs(r["achieved"] - 2.0 * 65536 ** 2 * 256 / 0.66e-3 / 1e12) < 0.1
    assert abs(r["frac"] - r["achieved"] / 5000.0) < 1e-4


def test_division_critical_path():
    b = _bench()
    macs = np.array([1e8, 4.66e8, 2e8])
    cp = b.critical_path(macs, 0.40)
    per_cu = 5000e12 / 2 / 256          # MAC/s at one CU's share of the int8 peak
    assert cp["largest_division_macs"] == 4.66e8
    assert abs(cp["at_one_cu_peak_us"] - 4.66e8 / per_cu * 1e6) < 0.1
    assert abs(cp["frac_of_call"] - cp["at_one_cu_peak_us"] / 400.0) < 1e-3


def test_traffic_json_fields():
    # the stored counters carry their commands and both calibrations
    t = json.load(open(os.path.join(ROOT, "profiles", "mfma_mul_2e19_traffic.json")))
    for k in ("kernel_sha", "fetch_size_kib_per_dispatch", "write_size_kib_per_dispatch",
              "fetch_scale_from_copy", "write_scale_from_copy", "bytes_per_launch", "commands"):
        assert k in t, k
    want = (t["fetch_size_kib_per_dispatch"] * t["fetch_scale_from_copy"] +
            t["write_size_kib_per_dispatch"] * t["write_scale_from_copy"]) * 1024
    assert abs(t["bytes_per_launch"] - want) <= 1024
    assert all(c.startswith("rocprofv3 --pmc ") for c in t["commands"])


def test_source_sha_names_the_sources():
    b = _bench()
    h = b.source_sha()
    assert len(h) == 16 and all(c in "0123456789abcdef" for c in h)
    assert h == b.source_sha()


def test_traffic_only_for_the_kernel_it_was_taken_on(tmp_path):
    # stored counters count for the kernel sources they were taken on; other
    # sources, or no record at all, give null traffic
    b = _bench()
    path = os.path.join(ROOT, "profiles", "mfma_mul_2e19_traffic.json")
    t = json.load(open(path))
    assert b.stored_traffic(path, t["kernel_sha"]) == t["bytes_per_launch"]
    assert b.stored_traffic(path, "0" * 16) is None
    assert len(b.kernel_sha()) == 16
    assert b.stored_traffic(str(tmp_path / "none.json"), b.kernel_sha()) is None
