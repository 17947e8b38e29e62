#!/usr/bin/env python
"""Throughput of the AT Burgers stepper on one MI355X.

One "step" of this benchmark is one complete run of the headline workload:
1D viscous Burgers, N = 2^24 points, P = 4096 tiles, 4th-order AT schemes,
L = 4 (k = 0 w.p. 1/2 else U{1..4}), nu = 1e-3, 2000 time steps, starting
from the seeded kappa^-2 field already resident in HBM.  The value is grid-point
updates per second (N * 2000 per step).  The same JSON line carries the
roofline of the dominant kernel, the CPU oracle timed on a bounded sample, and
sub-measurements of the plain one-launch-per-step form, the adjoint, the
batched form and the 3D vector stepper.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--only main|all]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E
FP64_ADDMUL_PEAK_TFLOPS = 39.3  # 256 CU x 64 FP64 lanes/clk x 2.4 GHz, one op per add or mul
METRIC = "grid-point updates/s & % HBM peak (AT step, adjoint, batched) vs plain form"


def eprint(*a):
    print(*a, file=sys.stderr, flush=True)


def flops_per_update(order):
    # stencil + update without contraction: order 2: 11, order 4: 17
    return 11 if order == 2 else 17


def algo_bytes_1d(N, P, order, L, dist, s):
    """Algorithmic HBM bytes of one launch advancing s steps: the field in and
    out once, plus per step the ring publish (2P*h doubles), the expected
    delayed-edge reads (m levels for faces with k > 0) and the delay row."""
    h = order // 2
    m = 2 if order == 2 else 3
    pk = (L / (L + 1.0)) if dist == 0 else (0.5 if L > 0 else 0.0)
    per_step = 2 * P * h * 8 + 2 * P * h * 8 * m * pk + 2 * P
    return 16.0 * N + s * per_step


class Timer:
    """HIP events on the stream the library launches on (torch's current stream)."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = []

    def start(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.pairs.append([e, None])

    def stop(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.pairs[-1][1] = e

    def total_ms(self):
        self.torch.cuda.synchronize()
        return sum(a.elapsed_time(b) for a, b in self.pairs)


def bench_c2(args, torch, at, I, fuse=None, label="main"):
    wl = I.wl_powerlaw_1d()
    N, P = wl.n[0], wl.p[0]
    st = at.Stepper(n=N, p=P, order=wl.order, L=wl.L, nu=wl.nu, dt=wl.dt, nsteps_max=wl.nsteps,
                    seed=wl.seed, dist=wl.dist)
    u0 = torch.from_numpy(wl.u0).cuda()
    if fuse is None:
        s = st.autotune(u0, 100)
    else:
        st.set_fuse(fuse)
        s = fuse
    snap = st.snapshot(u0)
    u = torch.empty_like(u0)
    scr = torch.empty_like(u0)
    for _ in range(args.warmup):
        st.restore(snap, u)
        st.run(u, scr, wl.nsteps)
    tm = Timer(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        st.restore(snap, u)
        tm.start()
        st.run(u, scr, wl.nsteps)
        tm.stop()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = tm.total_ms()
    launches = math.ceil(wl.nsteps / s)
    ms_launch = kern_ms / (args.steps * launches)
    # the last launch of a run may carry fewer steps; use the mean steps per launch
    s_mean = wl.nsteps / launches
    bytes_launch = algo_bytes_1d(N, P, wl.order, wl.L, wl.dist, s_mean)
    flops_launch = flops_per_update(wl.order) * N * s_mean
    gbps = bytes_launch / (ms_launch * 1e-3) / 1e9
    tflops = flops_launch / (ms_launch * 1e-3) / 1e12
    res = dict(wl=wl, s=s, wall=wall, ms_per_step=wall * 1e3 / args.steps,
               value=N * wl.nsteps * args.steps / wall, ms_launch=ms_launch, gbps=gbps,
               tflops=tflops, launches=launches, bytes_launch=bytes_launch, u0=wl.u0,
               delays=st.delays(), uT=u)
    eprint("[%s] fuse %d: %.3f ms/run, %.4g updates/s, kernel %.1f us/launch, %.0f GB/s, "
           "%.2f TFLOP/s" % (label, s, res["ms_per_step"], res["value"], ms_launch * 1e3, gbps,
                             tflops))
    return res


def roofline(r):
    hbm = dict(bound="hbm", achieved=round(r["gbps"], 2), peak=HBM_PEAK_GBPS, unit="GB/s",
               frac=round(r["gbps"] / HBM_PEAK_GBPS, 4), traffic=None)
    alu = dict(bound="alu", achieved=round(r["tflops"], 4), peak=FP64_ADDMUL_PEAK_TFLOPS,
               unit="TFLOP/s", frac=round(r["tflops"] / FP64_ADDMUL_PEAK_TFLOPS, 4),
               traffic=None)
    return (hbm, alu) if hbm["frac"] >= alu["frac"] else (alu, hbm)


def cpu_baseline(res):
    import numpy as np
    import oracle
    wl = res["wl"]
    N, P = wl.n[0], wl.p[0]
    k = res["delays"]
    t0 = time.perf_counter()
    oracle.run1d(wl.u0, N, P, wl.order, wl.L, wl.nu, wl.dt, k, 2)
    probe = time.perf_counter() - t0
    steps = int(max(2, min(wl.nsteps, round(12.0 / max(probe / 2, 1e-6)))))
    t0 = time.perf_counter()
    oracle.run1d(wl.u0, N, P, wl.order, wl.L, wl.nu, wl.dt, k, steps)
    el = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    eprint("[cpu] oracle %d steps in %.2f s on %d threads" % (steps, el, cores))
    return dict(value=N * steps / el, unit="grid-point updates/s", cores=cores, kind="oracle",
                sample="first %d of the 2000 steps of the same workload (N=2^24, P=4096, "
                       "order 4, same u0 and delays), %.1f s wall" % (steps, el))


def calibrate(torch):
    """Plain device copy of a known size: 2^27 doubles (1 GiB) read and written
    per launch, 5 launches, for scaling the HBM byte counters."""
    n = 1 << 27
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    tm = Timer(torch)
    for _ in range(5):
        tm.start()
        dst.copy_(src)
        tm.stop()
    ms = tm.total_ms() / 5
    eprint("[calibrate] copy of %d bytes: %.3f ms, %.1f GB/s (read+write)" %
           (8 * n, ms, 16.0 * n / (ms * 1e-3) / 1e9))
    print(json.dumps({"calibration_bytes_read": 8 * n, "calibration_bytes_written": 8 * n,
                      "ms_per_copy": ms}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--only", choices=["main", "all"], default="all")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fuse", type=int, default=None,
                    help="steps per launch of the headline run (default: autotuned)")
    ap.add_argument("--calibrate", action="store_true",
                    help="only copy 1 GiB of doubles 5 times (counter scale reference)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        eprint("bench.py: this build runs on one GPU only; the halo exchange of a "
               "multi-GPU run is a design note, not a measured path (asked for %d)" %
               max(args.gpus, world))
        sys.exit(2)
    import numpy as np  # noqa: F401
    import torch
    from paper_1911_05769_amd import at
    from paper_1911_05769_amd import inputs as I

    if not torch.cuda.is_available():
        eprint("bench.py: no GPU visible")
        sys.exit(1)
    at.lib()
    if args.calibrate:
        calibrate(torch)
        return
    main_res = bench_c2(args, torch, at, I, fuse=args.fuse)
    rl, rl_other = roofline(main_res)
    out = {
        "metric": METRIC,
        "value": main_res["value"],
        "unit": "grid-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_res["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": main_res["wl"].name, "n": main_res["wl"].n[0],
                   "p": main_res["wl"].p[0], "order": 4, "L": 4, "nsteps": 2000,
                   "fuse_steps": main_res["s"], "kernel": "k_step1d<4,false>"},
        "roofline": rl,
        "roofline_other": rl_other,
    }
    paths = {}
    if args.only == "all":
        plain = bench_c2(args, torch, at, I, fuse=1, label="plain")
        prl, _ = roofline(plain)
        paths["plain_1d"] = {"value": plain["value"], "unit": "grid-point updates/s",
                             "ms_per_step": round(plain["ms_per_step"], 4),
                             "kernel_us_per_launch": round(plain["ms_launch"] * 1e3, 3),
                             "hbm_gbps": round(plain["gbps"], 1),
                             "hbm_frac": round(plain["gbps"] / HBM_PEAK_GBPS, 4),
                             "fused_speedup": round(main_res["value"] / plain["value"], 3),
                             "bitwise_equal_to_fused": bool(torch.equal(plain["uT"],
                                                                        main_res["uT"]))}
        for name, fn in EXTRA:
            try:
                paths[name] = fn(args, torch, at, I)
            except Exception as e:   # reported, never hidden
                paths[name] = {"error": "%s: %s" % (type(e).__name__, e)}
                eprint("[%s] failed: %s" % (name, e))
    if paths:
        out["paths"] = paths
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(main_res)
    print(json.dumps(out), flush=True)


EXTRA = []

if __name__ == "__main__":
    main()
