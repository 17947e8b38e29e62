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

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, published
FP64_PEAK_TFLOPS = 78.6         # MI355X vector FP64, published (an FMA counts two flops)
FP64_ISSUE_TINSTR = 39.3        # 256 CU x 4 SIMD x 16 lanes x 2.4 GHz: FP64 VALU
                                # instructions per second (a wave64 instruction takes
                                # four cycles on a 16-lane SIMD)
METRIC = "grid-point updates/s & % HBM peak (AT step, adjoint, batched) vs plain form"

# HBM bytes per launch of the headline kernel, from rocprofv3 FETCH_SIZE x 2.0 +
# WRITE_SIZE x 1.0 (scales from a plain 1 GiB copy); reported only while the
# kernel source hashes to the value the counters were taken on, and null
# (bytes_per_launch None) until they have been taken on the current source.
TRAFFIC = {"sources": ["paper_1911_05769_amd/csrc/at_step1d.hip",
                       "paper_1911_05769_amd/csrc/at_stencil1d.h"],
           "md5": "1a8eca99f62c6fbc1b646766206a9922", "fuse": 56,
           # FETCH_SIZE 73249.3 KiB x 2.0 + WRITE_SIZE 132608.0 KiB x 1.0, mean of the 35
           # 56-step launches of one 2000-step run
           "bytes_per_launch": 285805158.4}


def eprint(*a):
    print(*a, file=sys.stderr, flush=True)


def flops_per_update(order, arith=0):
    """(flops, FP64 VALU instructions) of one interior update.  The flops are
    the method's own (section 3.2's central differences and the Euler update):
    11 for order 2, 17 for order 4, in every arithmetic mode.  Instructions:
    exact order issues order 2 in 10 and order 4 in 15 (the exact scalings by
    2, 8 and 16 share an fma with the next add, one rounding either way); the
    contracted mode issues order 2 in 6 and order 4 in 10."""
    if arith == 0:
        return (11, 10) if order == 2 else (17, 15)
    return (11, 6) if order == 2 else (17, 10)


def algo_bytes_1d(N, P, order, L, dist, s):
    """Algorithmic HBM bytes of one launch advancing s steps: the field in and
    out once, the delay rows (2P bytes per step), and the ring traffic.  One
    step per launch reads the delayed edge levels it uses from the ring (m
    levels of the faces with k > 0) and publishes its level; a fused launch
    copies the D = L + m - 1 edge levels below its first step into LDS once,
    takes every later delayed level from there, and publishes only its last
    min(s, D) levels (the ones the next launch reads)."""
    h = order // 2
    m = 2 if order == 2 else 3
    D = L + m - 1
    edge_level = 2 * P * h * 8                       # one level of every tile edge
    if s == 1:
        pk = (L / (L + 1.0)) if dist == 0 else (0.5 if L > 0 else 0.0)
        ring = edge_level + edge_level * m * pk
    else:
        ring = edge_level * D + edge_level * min(s, D)
    return 16.0 * N + ring + s * 2 * P


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

    def each_ms(self):
        self.torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in self.pairs]


def spread(ms):
    """median and interquartile range of per-run times (ms)"""
    import numpy as np
    q1, med, q3 = np.percentile(np.asarray(ms, dtype=np.float64), [25, 50, 75])
    return {"runs": len(ms), "median_ms": round(float(med), 4),
            "iqr_ms": [round(float(q1), 4), round(float(q3), 4)],
            "min_ms": round(float(min(ms)), 4), "max_ms": round(float(max(ms)), 4)}


def bench_c2(args, torch, at, I, fuse=None, label="main", arith=0):
    wl = I.wl_powerlaw_1d()
    N, P = wl.n[0], wl.p[0]
    st = at.Stepper(n=N, p=P, order=wl.order, L=wl.L, nu=wl.nu, dt=wl.dt, nsteps_max=wl.nsteps,
                    seed=wl.seed, dist=wl.dist, arith=arith)
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
    run_ms = tm.each_ms()
    launches = math.ceil(wl.nsteps / s)
    ms_launch = kern_ms / (args.steps * launches)
    # the last launch of a run may carry fewer steps; use the mean steps per launch
    s_mean = wl.nsteps / launches
    bytes_launch = algo_bytes_1d(N, P, wl.order, wl.L, wl.dist, s_mean)
    fl, ins = flops_per_update(wl.order, arith)
    flops_launch = fl * N * s_mean
    gbps = bytes_launch / (ms_launch * 1e-3) / 1e9
    tflops = flops_launch / (ms_launch * 1e-3) / 1e12
    # issue-rate ceiling for this instruction mix: 39.3 T FP64 instructions/s
    # (a diagnostic; the roofline's peak is the published 78.6 TFLOP/s)
    issue_ceiling = FP64_ISSUE_TINSTR * fl / ins
    # one step per launch runs the plain kernel (8 points per thread)
    ppt = 8 if s == 1 else {1: 16, 2: 8, 3: 4}.get(st.variant, 16)
    res = dict(wl=wl, s=s, ppt=ppt, wall=wall, ms_per_step=wall * 1e3 / args.steps, run_ms=run_ms,
               value=N * wl.nsteps * args.steps / wall, ms_launch=ms_launch, gbps=gbps,
               tflops=tflops, issue_ceiling=issue_ceiling, arith=arith, launches=launches,
               bytes_launch=bytes_launch, u0=wl.u0,
               delays=st.delays(), uT=u)
    eprint("[%s] fuse %d, %d points/thread: %.3f ms/run, %.4g updates/s, kernel %.1f us/launch, "
           "%.0f GB/s, %.2f TFLOP/s" % (label, s, ppt, res["ms_per_step"], res["value"],
                                        ms_launch * 1e3, gbps, tflops))
    st.close()
    return res


def sources_md5(paths):
    import hashlib
    h = hashlib.md5()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(r):
    """Counter-measured HBM bytes per launch, or None when they do not apply
    (no counters taken on the current source, another steps-per-launch, or
    the contracted arithmetic)."""
    if TRAFFIC["md5"] is None or TRAFFIC["bytes_per_launch"] is None:
        return None
    try:
        md5 = sources_md5(TRAFFIC["sources"])
    except OSError:
        return None
    if md5 != TRAFFIC["md5"] or r["s"] != TRAFFIC["fuse"] or r.get("arith", 0) != 0:
        return None
    return round(TRAFFIC["bytes_per_launch"])


def roofline(r):
    """(dominant, other): the HBM roofline (algorithmic bytes per launch over
    the launch time, against 8 TB/s) and the FP64 one (the update's flops per
    launch over the launch time, against the published 78.6 TFLOP/s); the
    dominant one is the larger fraction.  The FP64 entry also carries the
    issue ceiling of the kernel's instruction mix as a diagnostic."""
    traffic = measured_traffic(r)
    hbm = dict(bound="hbm", achieved=round(r["gbps"], 2), peak=HBM_PEAK_GBPS, unit="GB/s",
               frac=round(r["gbps"] / HBM_PEAK_GBPS, 4), traffic=traffic)
    alu = dict(bound="alu", achieved=round(r["tflops"], 4), peak=FP64_PEAK_TFLOPS,
               unit="TFLOP/s", frac=round(r["tflops"] / FP64_PEAK_TFLOPS, 4), traffic=traffic,
               issue_ceiling_tflops=round(r["issue_ceiling"], 2),
               frac_of_issue_ceiling=round(r["tflops"] / r["issue_ceiling"], 4))
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
    # the 2-step probe carries start-up costs: aim it at ~30 s for ~10-15 s of work
    steps = int(max(2, min(wl.nsteps, round(30.0 / max(probe / 2, 1e-6)))))
    t0 = time.perf_counter()
    oracle.run1d(wl.u0, N, P, wl.order, wl.L, wl.nu, wl.dt, k, steps)
    el = time.perf_counter() - t0
    cores = oracle.max_threads()
    eprint("[cpu] oracle %d steps in %.2f s on %d threads" % (steps, el, cores))
    # one thread, a shorter sample of the same steps
    steps1 = max(2, min(steps, int(round(8.0 / max(el * cores / steps, 1e-6)))))
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.run1d(wl.u0, N, P, wl.order, wl.L, wl.nu, wl.dt, k, steps1)
    el1 = time.perf_counter() - t0
    oracle.set_threads(cores)
    eprint("[cpu] oracle %d steps in %.2f s on 1 thread" % (steps1, el1))
    return dict(value=N * steps / el, unit="grid-point updates/s", cores=cores, kind="oracle",
                sample="first %d of the 2000 steps of the same workload (N=2^24, P=4096, "
                       "order 4, same u0 and delays), %.1f s wall" % (steps, el),
                value_1thread=N * steps1 / el1, sample_1thread="first %d steps, %.1f s" %
                (steps1, el1), host=host_info())


def host_info():
    info = {"nproc": os.cpu_count()}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    info["ram_gb"] = round(int(line.split()[1]) / 2 ** 20, 1)
                    break
    except OSError:
        pass
    return info


def copy_ceiling(torch, n=1 << 27, reps=5):
    """Achieved rate of torch's device copy of n doubles (read + write; the
    runtime's device-to-device copy), on the same stream and with the same
    events as the kernels.  The library's own copy kernel streams faster
    (copy_ceiling_lib)."""
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    tm = Timer(torch)
    for _ in range(reps):
        tm.start()
        dst.copy_(src)
        tm.stop()
    ms = tm.total_ms() / reps
    del src, dst
    return ms, 16.0 * n / (ms * 1e-3) / 1e9


def copy_ceiling_lib(torch, at, n=1 << 27, reps=5):
    """The library's own device copy (at_restore of a 2^27-point state: the
    field and a small ring), timed the same way as copy_ceiling.  It streams
    faster than the runtime's device-to-device copy that copy_ceiling uses."""
    st = at.Stepper(n=n, p=1024, order=2, L=0, nu=1e-3, dt=1e-6, nsteps_max=1, seed=1)
    u = torch.ones(n, dtype=torch.float64, device="cuda")
    snap = st.snapshot(u)
    st.restore(snap, u)
    tm = Timer(torch)
    for _ in range(reps):
        tm.start()
        st.restore(snap, u)
        tm.stop()
    ms = tm.total_ms() / reps
    st.close()
    del st, u, snap
    return ms, 16.0 * n / (ms * 1e-3) / 1e9


def calibrate(torch):
    """Plain device copy of a known size: 2^27 doubles (1 GiB) read and written
    per launch, 5 launches, for scaling the HBM byte counters."""
    n = 1 << 27
    ms, _ = copy_ceiling(torch, n)
    eprint("[calibrate] copy of %d bytes: %.3f ms, %.1f GB/s (read+write)" %
           (8 * n, ms, 16.0 * n / (ms * 1e-3) / 1e9))
    print(json.dumps({"calibration_bytes_read": 8 * n, "calibration_bytes_written": 8 * n,
                      "ms_per_copy": ms}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=15)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--only", choices=["main", "all"], default="all")
    ap.add_argument("--legs", default="plain,contracted,c1,batched,adjoint,3d,scalars,ws",
                    help="comma-separated sub-measurements run with --only all")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fuse", type=int, default=None,
                    help="steps per launch of the headline run (default: autotuned)")
    ap.add_argument("--batch-fuse", type=int, default=None,
                    help="batched leg: steps per launch at 16 points per thread (default: autotuned)")
    ap.add_argument("--variant3d", type=int, default=None,
                    help="3D legs: run this kernel variant instead of the autotuned one")
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
                   "fuse_steps": main_res["s"], "points_per_thread": main_res["ppt"],
                   "arith": "exact order, no contraction",
                   "kernel": ("k_step1d_plain<4,false,false>" if main_res["s"] == 1
                              else "k_step1d_aligned<4,false,false,%d>" % main_res["ppt"])},
        "roofline": rl,
        "roofline_other": rl_other,
        "timing": dict(spread(main_res["run_ms"]), clock="HIP events around each 2000-step run"),
    }
    paths = {}
    legs = set(x.strip() for x in args.legs.split(",") if x.strip())
    if args.only == "all" and "plain" in legs:
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
    if args.only == "all" and "contracted" in legs:
        con = bench_c2(args, torch, at, I, label="contracted", arith=1)
        crl, _ = roofline(con)
        import numpy as np
        a = main_res["uT"].cpu().numpy()
        b = con["uT"].cpu().numpy()
        paths["contracted_1d"] = {
            "value": con["value"], "unit": "grid-point updates/s",
            "ms_per_step": round(con["ms_per_step"], 4), "fuse_steps": con["s"],
            "kernel_us_per_launch": round(con["ms_launch"] * 1e3, 3),
            "roofline": crl,
            "speedup_vs_exact_order": round(con["value"] / main_res["value"], 3),
            "max_rel_diff_vs_exact_order_after_2000_steps":
                float(np.max(np.abs(a - b)) / np.max(np.abs(a)))}
    if args.only == "all":
        for name, fn in EXTRA:
            if name not in legs:
                continue
            try:
                paths[name] = fn(args, torch, at, I)
            except Exception as e:   # reported, never hidden
                paths[name] = {"error": "%s: %s" % (type(e).__name__, e)}
                eprint("[%s] failed: %s" % (name, e))
    ms_copy, copy_gbps = copy_ceiling(torch)
    out["hbm_copy_gbps"] = round(copy_gbps, 1)
    eprint("[copy] 1 GiB device copy: %.3f ms, %.0f GB/s" % (ms_copy, copy_gbps))
    ms_lcopy, lcopy_gbps = copy_ceiling_lib(torch, at)
    out["hbm_copy_kernel_gbps"] = round(lcopy_gbps, 1)
    eprint("[copy] 1 GiB copy by the library's copy kernel: %.3f ms, %.0f GB/s" %
           (ms_lcopy, lcopy_gbps))
    if paths:
        out["paths"] = paths
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(main_res)
    print(json.dumps(out), flush=True)

def _timed(torch, fn):
    tm = Timer(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tm.start()
    fn()
    tm.stop()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, tm.total_ms() * 1e-3


def bench_batched(args, torch, at, I):
    """256 independent 1D instances (uneven N, nu, L, seeds), order 4, 500
    steps: (i) one launch per instance per step, (ii) one launch per step over
    all instances, (iii) the fused batched form replayed from a HIP graph."""
    wls = I.batch_instances()
    nst = wls[0].nsteps
    pts = sum(w.n[0] for w in wls)
    u0 = [torch.from_numpy(w.u0).cuda() for w in wls]
    us = [u.clone() for u in u0]
    ss = [torch.empty_like(u) for u in u0]
    res = {"instances": len(wls), "points": pts, "nsteps": nst}
    # (i) per-instance plain runs
    steppers = [at.Stepper(n=w.n[0], p=w.p[0], order=w.order, L=w.L, nu=w.nu, dt=w.dt,
                           nsteps_max=nst, seed=w.seed, dist=w.dist) for w in wls]
    snaps = [st.snapshot(u) for st, u in zip(steppers, u0)]

    def per_instance():
        for st, sn, u, s in zip(steppers, snaps, us, ss):
            st.restore(sn, u)
            st.run(u, s, nst)
    per_instance()
    w1, k1 = _timed(torch, per_instance)
    ref = [u.clone() for u in us]
    for st in steppers:
        st.close()
    del steppers, snaps
    # (ii) batched, one launch per step, no graph; (iii) fused + graph
    b = at.Batch.from_workloads(wls)

    def batched(use_graph):
        b.reset()
        for u, v in zip(us, u0):
            u.copy_(v)
        b.run(us, ss, nst, use_graph=use_graph)

    b.set_fuse(1)
    batched(False)
    w2, k2 = _timed(torch, lambda: batched(False))
    b.reset()
    if args.batch_fuse:
        b.set_variant(1)
        b.set_fuse(args.batch_fuse)
        s = args.batch_fuse
    else:
        s = b.autotune(u0, 128)
    batched(True)                       # capture
    reps = max(1, args.steps)
    tm = Timer(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.reset()
        for u, v in zip(us, u0):
            u.copy_(v)
        tm.start()
        b.run(us, ss, nst, use_graph=True)
        tm.stop()
    torch.cuda.synchronize()
    w3 = (time.perf_counter() - t0) / reps
    k3 = tm.total_ms() * 1e-3 / reps
    same = all(torch.equal(a, r) for a, r in zip(us, ref))
    upd = pts * nst
    algo = sum(algo_bytes_1d(w.n[0], w.p[0], w.order, w.L, w.dist, 1) for w in wls) * nst
    res.update({
        "value": upd / k3, "unit": "grid-point updates/s", "fuse_steps": s,
        "points_per_thread": {0: 16, 1: 16, 2: 8, 3: 4}[b.variant],
        "ms_graph_run": round(k3 * 1e3, 3),
        "ms_per_instance_plain": round(k1 * 1e3, 3),
        "ms_one_launch_per_step": round(k2 * 1e3, 3),
        "speedup_vs_per_instance": round(k1 / k3, 2),
        "speedup_vs_one_launch_per_step": round(k2 / k3, 2),
        "one_launch_per_step_hbm_gbps": round(algo / k2 / 1e9, 1),
        # the method's 17 flops per order-4 update against the published FP64 peak
        "fp64_tflops": round(17.0 * upd / k3 / 1e12, 3),
        "fp64_frac": round(17.0 * upd / k3 / 1e12 / FP64_PEAK_TFLOPS, 4),
        "bitwise_equal_to_per_instance": bool(same)})
    eprint("[batched] %d instances, %d points: per-instance %.1f ms, one launch/step %.1f ms, "
           "fused(s=%d, variant %d)+graph %.2f ms (%.3g updates/s)" %
           (len(wls), pts, k1 * 1e3, k2 * 1e3, s, b.variant, k3 * 1e3, upd / k3))
    b.close()
    return res


def bench_adjoint(args, torch, at, I):
    """Gradient of 0.5||u(T) - u_target||^2 w.r.t. u0 (2^20 values) and nu for
    4000 steps, order 2, P = 1024, L = 3, checkpoints every 100 steps."""
    wl = I.wl_adjoint_1d()
    N, P, nst, C = wl.n[0], wl.p[0], wl.nsteps, wl.extra["ckpt"]
    u0 = torch.from_numpy(wl.u0).cuda()
    scr = torch.empty_like(u0)
    tst = at.Stepper(n=N, p=P, order=2, L=wl.L, nu=wl.extra["nu_target"], dt=wl.dt,
                     nsteps_max=nst, seed=wl.seed, fuse_steps=32)
    target = u0.clone()
    tst.run(target, scr, nst)
    times = []
    for rep in range(max(1, args.steps)):
        st = at.Stepper(n=N, p=P, order=2, L=wl.L, nu=wl.nu, dt=wl.dt, nsteps_max=nst,
                        seed=wl.seed, record=True, ckpt_every=C, fuse_steps=32)
        u = u0.clone()
        lam = torch.empty_like(u)
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        st.run(u, scr, nst)
        J = st.loss(u, target, lam)
        ev[1].record()
        g, gnu = st.adjoint(lam)
        ev[2].record()
        torch.cuda.synchronize()
        times.append((ev[0].elapsed_time(ev[1]) * 1e-3, ev[1].elapsed_time(ev[2]) * 1e-3))
        st.close()
    tst.close()
    tf = min(t[0] for t in times)
    ta = min(t[1] for t in times)
    pstep = N * nst
    # reverse sweep, algorithmic floor: every intermediate level of u is written
    # once by the recompute and read once by the reverse steps (16 B per
    # point-step); lambda stays on chip within a fused reverse launch
    gbps = pstep * 16.0 / ta / 1e9
    eprint("[adjoint] forward %.2f ms, adjoint %.2f ms (%.0f GB/s algorithmic), J %.3e, "
           "dJ/dnu %.4e" % (tf * 1e3, ta * 1e3, gbps, float(J), float(gnu)))
    return {"value": pstep / (tf + ta), "unit": "point-steps/s (gradient)",
            "ms_forward_recorded": round(tf * 1e3, 3), "ms_adjoint": round(ta * 1e3, 3),
            "adjoint_hbm_gbps": round(gbps, 1), "adjoint_hbm_frac": round(gbps / HBM_PEAK_GBPS, 4),
            "n": N, "nsteps": nst, "ckpt_every": C}


def bench_c1(args, torch, at, I):
    """The small correctness configuration: N = 1024, P = 8, order 2, L = 2,
    1000 steps (8 KB of state: launch-latency bound).  Microseconds per step
    for one launch per step and for the autotuned steps per launch, each with
    launches issued one by one and replayed from a captured HIP graph, and for
    the whole grid in one workgroup (one launch per run)."""
    wl = I.wl_sines_1d()
    N, P = wl.n[0], wl.p[0]
    u0 = torch.from_numpy(wl.u0).cuda()
    out = {"workload": wl.name}
    uT = {}
    for label, fuse, graph in (("plain", 1, False), ("plain_graph", 1, True),
                               ("fused", 0, False), ("fused_graph", 0, True),
                               ("single_workgroup", -1, False)):
        st = at.Stepper(n=N, p=P, order=2, L=wl.L, nu=wl.nu, dt=wl.dt, nsteps_max=wl.nsteps,
                        seed=wl.seed, dist=wl.dist)
        if fuse == 0:
            fuse = st.autotune(u0, 100)
        elif fuse < 0:
            st.set_variant(4)                 # the whole grid in one workgroup
            fuse = st.query()[1]
        else:
            st.set_fuse(fuse)
        st.set_graph(graph)
        snap = st.snapshot(u0)
        u, s = torch.empty_like(u0), torch.empty_like(u0)
        st.restore(snap, u)
        st.run(u, s, wl.nsteps)
        tm = Timer(torch)
        for _ in range(max(3, args.steps)):
            st.restore(snap, u)
            tm.start()
            st.run(u, s, wl.nsteps)
            tm.stop()
        sp = spread(tm.each_ms())
        uT[label] = u.clone()
        us = sp["median_ms"] * 1e3 / wl.nsteps
        eprint("[c1] %s (s=%d): %.3f us/step" % (label, fuse, us))
        out[label] = {"fuse_steps": fuse, "us_per_step": round(us, 3), "timing": sp,
                      "graph_replay": graph}
        st.close()
    out["bitwise_equal"] = all(bool(torch.equal(uT["plain"], uT[x]))
                               for x in ("plain_graph", "fused", "fused_graph",
                                         "single_workgroup"))
    # the weakly-synchronous run: 8 one-wave workgroups, emergent delays
    import numpy as np
    ws_ms, hist = [], None
    for rep in range(max(3, args.steps) + 1):
        st = at.Stepper(n=N, p=P, order=2, L=wl.L, nu=wl.nu, dt=wl.dt, nsteps_max=wl.nsteps,
                        seed=wl.seed, dist=wl.dist)
        u = u0.clone()
        tm = Timer(torch)
        tm.start()
        st.run_ws(u, wl.nsteps)
        tm.stop()
        if rep > 0:
            ws_ms.append(tm.total_ms())
            hist = np.bincount(st.delays()[:wl.nsteps].ravel().astype(np.int64),
                               minlength=wl.L + 1)
    sp = spread(ws_ms)
    us = sp["median_ms"] * 1e3 / wl.nsteps
    frac = (hist / hist.sum()).round(4).tolist()
    eprint("[c1] weakly-synchronous (emergent delays): %.3f us/step, delays k=0..%d: %s" %
           (us, wl.L, frac))
    out["weakly_synchronous"] = {"us_per_step": round(us, 3), "timing": sp,
                                 "delay_fractions": frac}
    out["value"] = min(out[x]["us_per_step"] for x in ("plain", "plain_graph", "fused",
                                                       "fused_graph", "single_workgroup"))
    out["unit"] = "us/step (lower is better)"
    return out


def bench_ws(args, torch, at, I):
    """Weakly-synchronous runs with emergent delays (one workgroup per tile or
    block, no global barrier, level counters): 1D N = 2^20, 1024 tiles of 1024
    points, order 2, 2000 steps, and 3D 512^3 with 8^3 blocks, 200 steps;
    L = 3 against L = 0 (every step waits for its neighbours: the
    synchronous algorithm), and the prescribed-delay path on the same grids."""
    import numpy as np
    wl = I.wl_adjoint_1d()
    N, P, nst = wl.n[0], wl.p[0], 2000
    u0 = torch.from_numpy(wl.u0).cuda()
    out = {"n": N, "p": P, "nsteps": nst}
    # jitter J: before each step a tile idles a pseudo-random 0..J units of
    # about 128 clocks (uneven arrival, as network noise causes)
    for jitter in (0, 32):
        for L in (3, 0):
            best, hist = None, None
            for rep in range(max(1, min(args.steps, 3)) + 1):
                st = at.Stepper(n=N, p=P, order=2, L=L, nu=wl.nu, dt=wl.dt, nsteps_max=nst,
                                seed=wl.seed)
                u = u0.clone()
                tm = Timer(torch)
                tm.start()
                st.run_ws(u, nst, jitter=jitter, seed=rep)
                tm.stop()
                ms = tm.total_ms()
                if rep > 0 and (best is None or ms < best):      # the first run warms up
                    best = ms
                    hist = np.bincount(st.delays()[:nst].ravel().astype(np.int64),
                                       minlength=L + 1)
                st.close()
            frac = (hist / hist.sum()).round(4).tolist()
            eprint("[ws] jitter %d, L=%d: %.2f ms/run (%.2f us/step), delays k=0..%d: %s" %
                   (jitter, L, best, best * 1e3 / nst, L, frac))
            out["ws_L%d_jitter%d" % (L, jitter)] = {
                "ms_per_run": round(best, 3), "us_per_step": round(best * 1e3 / nst, 3),
                "updates_per_s": N * nst / (best * 1e-3), "delay_fractions": frac}
    st = at.Stepper(n=N, p=P, order=2, L=3, nu=wl.nu, dt=wl.dt, nsteps_max=nst, seed=wl.seed)
    fuse = st.autotune(u0, 64)
    u, s = u0.clone(), torch.empty_like(u0)
    snap = st.snapshot(u0)
    st.restore(snap, u)
    st.run(u, s, nst)
    tm = Timer(torch)
    reps = max(1, min(args.steps, 3))
    for _ in range(reps):
        st.restore(snap, u)
        tm.start()
        st.run(u, s, nst)
        tm.stop()
    ms = tm.total_ms() / reps
    eprint("[ws] prescribed delays, fused s=%d: %.2f ms/run" % (fuse, ms))
    out["prescribed_L3"] = {"ms_per_run": round(ms, 3), "fuse_steps": fuse,
                            "updates_per_s": N * nst / (ms * 1e-3)}
    st.close()
    # 3D: 512^3 x 3, 8^3 blocks of 64^3, one resident workgroup per block
    w3 = I.wl_solenoidal_3d()
    nst3 = w3.nsteps
    v0 = torch.from_numpy(w3.u0).cuda()
    v, s3 = torch.empty_like(v0), torch.empty_like(v0)
    npt3 = w3.npoints
    for L in (3, 0):
        best, hist = None, None
        for rep in range(max(1, min(args.steps, 2)) + 1):
            st = at.Stepper(dim=3, n=w3.n, p=w3.p, order=2, L=L, nu=w3.nu, dt=w3.dt,
                            nsteps_max=nst3, seed=w3.seed)
            v.copy_(v0)
            tm = Timer(torch)
            tm.start()
            st.run_ws(v, nst3, scratch=s3)
            tm.stop()
            ms = tm.total_ms()
            if rep > 0 and (best is None or ms < best):
                best = ms
                hist = np.bincount(st.delays()[:nst3].ravel().astype(np.int64), minlength=L + 1)
            st.close()
        frac = (hist / hist.sum()).round(4).tolist()
        eprint("[ws] 3D L=%d: %.1f ms/run (%.3f ms/step), delays k=0..%d: %s" %
               (L, best, best / nst3, L, frac))
        out["ws3d_L%d" % L] = {"ms_per_run": round(best, 3), "ms_per_step": round(best / nst3, 4),
                              "point_updates_per_s": npt3 * nst3 / (best * 1e-3),
                              "delay_fractions": frac}
    st = at.Stepper(dim=3, n=w3.n, p=w3.p, order=2, L=3, nu=w3.nu, dt=w3.dt, nsteps_max=nst3,
                    seed=w3.seed)
    var = st.autotune(v0, 6)
    snap = st.snapshot(v0)
    st.restore(snap, v)
    st.run(v, s3, nst3)
    tm = Timer(torch)
    st.restore(snap, v)
    tm.start()
    st.run(v, s3, nst3)
    tm.stop()
    ms = tm.total_ms()
    eprint("[ws] 3D prescribed delays, variant %d: %.1f ms/run" % (var, ms))
    out["prescribed3d_L3"] = {"ms_per_run": round(ms, 3), "kernel_variant": var}
    st.close()
    out["value"] = out["ws_L3_jitter0"]["updates_per_s"]
    out["unit"] = "grid-point updates/s (weakly-synchronous, emergent delays)"
    return out


def _bench_3d_run(args, torch, at, wl, alpha, tag):
    """Autotuned kernel variant, then whole runs of wl.nsteps steps timed from a
    restored snapshot; algorithmic bytes per point-update: NC = 3 + scalars
    components in and out (16 NC B) plus the ring (publish 6 faces of NC
    components; read levels n-k and n-k-1 of the faces with k > 0, a fraction
    L/(L+1) of them under uniform delays)."""
    nc = 3 + len(alpha)
    st = at.Stepper(dim=3, n=wl.n, p=wl.p, order=2, L=wl.L, nu=wl.nu, dt=wl.dt,
                    nsteps_max=wl.nsteps, seed=wl.seed, dist=wl.dist, alpha=alpha)
    u0 = torch.from_numpy(wl.u0).cuda()
    if args.variant3d is None:
        var = st.autotune(u0, 6)
    else:
        st.set_variant(args.variant3d)
        var = args.variant3d
    snap = st.snapshot(u0)
    u = torch.empty_like(u0)
    s = torch.empty_like(u0)
    st.restore(snap, u)
    st.run(u, s, wl.nsteps)
    reps = max(1, min(args.steps, 3))
    tm = Timer(torch)
    for _ in range(reps):
        st.restore(snap, u)
        tm.start()
        st.run(u, s, wl.nsteps)
        tm.stop()
    sec = tm.total_ms() * 1e-3 / reps
    npt = wl.npoints
    bx = wl.n[0] // wl.p[0]
    face_frac = 6.0 / bx
    ring_b = face_frac * 8.0 * nc * (1 + 2 * wl.L / (wl.L + 1.0))
    bpu = 16.0 * nc + ring_b
    gbps = npt * wl.nsteps * bpu / sec / 1e9
    st.close()
    eprint("[%s] variant %d" % (tag, var))
    eprint("[%s] %s: %.2f ms/run, %.3g point-updates/s, %.0f GB/s (%.1f B/update)" %
           (tag, wl.name, sec * 1e3, npt * wl.nsteps / sec, gbps, bpu))
    return {"value": npt * wl.nsteps / sec, "unit": "point-updates/s (%d components)" % nc,
            "ms_per_run": round(sec * 1e3, 3), "hbm_gbps": round(gbps, 1),
            "hbm_frac": round(gbps / HBM_PEAK_GBPS, 4), "bytes_per_update": round(bpu, 2),
            "workload": wl.name, "kernel_us_per_step": round(sec * 1e6 / wl.nsteps, 2),
            "kernel_variant": var}


def bench_3d(args, torch, at, I):
    """3D vector Burgers, 512^3 x 3 components, 8^3 blocks of 64^3, order 2,
    L = 3, 200 steps."""
    return _bench_3d_run(args, torch, at, I.wl_solenoidal_3d(), (), "3d")


def bench_scalars(args, torch, at, I):
    """3D vector Burgers with two passive scalars (Schmidt numbers 1 and 2),
    512^3 x 5 components, 8^3 blocks of 64^3, order 2, L = 3, 200 steps."""
    wl = I.wl_scalars_3d()
    return _bench_3d_run(args, torch, at, wl, wl.extra["alpha"], "scalars")


EXTRA = [("c1", bench_c1), ("batched", bench_batched), ("adjoint", bench_adjoint),
         ("3d", bench_3d), ("scalars", bench_scalars), ("ws", bench_ws)]

if __name__ == "__main__":
    main()
