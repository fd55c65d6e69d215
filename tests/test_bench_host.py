"""Host-side logic of bench.py that needs no GPU."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_summary_read_only_for_matching_kernel_source(tmp_path):
    b = _bench()
    # the committed summary matches the committed kernel source
    assert b.measured_traffic() is not None and b.measured_traffic() > 5e8
    text = open(b.TRAFFIC_SUMMARY).read()
    stale = tmp_path / "stale.md"
    stale.write_text(text.replace(b.kernel_source_hash(), "0000000000000000"))
    b.TRAFFIC_SUMMARY = str(stale)
    assert b.measured_traffic() is None
    b.TRAFFIC_SUMMARY = str(tmp_path / "missing.md")
    assert b.measured_traffic() is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
