"""Host-side checks of bench.py's contract (no GPU): a run asked for more than
one GPU exits with a message before touching any device, and the HBM byte
counts it reports for the headline kernel belong to the committed source."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_contract", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_counter_bytes_match_the_committed_kernel_source():
    """roofline.traffic is reported only while the hashed sources are the ones
    the counters were taken on; the stored hash must be the current one."""
    b = _bench_module()
    assert b.sources_md5(b.TRAFFIC["sources"]) == b.TRAFFIC["md5"]
    assert b.TRAFFIC["bytes_per_launch"] > 0
