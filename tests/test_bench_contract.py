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


def test_counter_bytes_only_for_the_measured_kernel_source():
    """roofline.traffic is reported only while the hashed sources are the ones
    the counters were taken on, for the same steps per launch and the exact
    arithmetic; otherwise it is null."""
    b = _bench_module()
    cur = b.sources_md5(b.TRAFFIC["sources"])
    r = {"s": b.TRAFFIC["fuse"], "arith": 0}
    saved = dict(b.TRAFFIC)
    try:
        b.TRAFFIC.update(md5=cur, bytes_per_launch=123456.0)
        assert b.measured_traffic(r) == 123456
        assert b.measured_traffic(dict(r, s=r["s"] + 1)) is None
        assert b.measured_traffic(dict(r, arith=1)) is None
        b.TRAFFIC.update(md5="0" * 32)
        assert b.measured_traffic(r) is None
    finally:
        b.TRAFFIC.clear()
        b.TRAFFIC.update(saved)
    if saved["md5"] is not None:        # stored counters belong to the current source
        assert saved["md5"] == cur and saved["bytes_per_launch"] > 0


def test_roofline_uses_published_peaks():
    b = _bench_module()
    r = {"s": 56, "arith": 0, "gbps": 530.0, "tflops": 29.4, "issue_ceiling": 44.5}
    dom, other = b.roofline(r)
    assert dom["bound"] == "alu" and dom["peak"] == 78.6
    assert abs(dom["frac"] - 29.4 / 78.6) < 1e-4
    assert other["bound"] == "hbm" and other["peak"] == 8000.0


def test_algorithmic_bytes_model():
    """One step per launch: field in and out, the level's edges published, the
    delayed edge levels read for the faces with k > 0, the delay row.  A
    fused launch: field once, D = L + m - 1 edge levels read into LDS and the
    last min(s, D) published, s delay rows."""
    b = _bench_module()
    N, P, L = 1 << 24, 4096, 4
    edge = 2 * P * 2 * 8                                   # order 4: h = 2
    plain = b.algo_bytes_1d(N, P, 4, L, 1, 1)
    assert plain == 16.0 * N + edge + edge * 3 * 0.5 + 2 * P
    fused = b.algo_bytes_1d(N, P, 4, L, 1, 56)
    assert fused == 16.0 * N + edge * 6 + edge * 6 + 56 * 2 * P
    assert b.algo_bytes_1d(N, P, 4, L, 1, 3) == 16.0 * N + edge * 6 + edge * 3 + 3 * 2 * P
    assert b.algo_bytes_1d(1024, 8, 2, 2, 0, 1) == 16.0 * 1024 + 16 * 8 + 16 * 8 * 2 * (2 / 3) + 16
