"""Batched form: many independent 1D instances of uneven size in shared
launches.  Every instance must equal the same instance run alone (bit for
bit) and the CPU oracle (<= 1e-12 normwise); graph replays must equal the
eager launch sequence on every replay."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1911_05769_amd import inputs as I

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def small_instances(nsteps=120):
    g = np.random.default_rng(4)
    out = []
    for j, (n, p) in enumerate([(512, 2), (1024, 8), (4096, 16), (768, 3), (2048, 4),
                                (8192, 32), (256, 1), (12288, 48)]):
        nu = float(g.uniform(1e-3, 5e-2))
        L = int(g.choice([1, 2, 4]))
        u0 = I.u0_powerlaw(n, n // 16, 300 + j)
        dt = I.dt_rule(2 * math.pi / n, float(np.max(np.abs(u0))), nu)
        out.append(I.Workload("s%d" % j, 1, (n, 1, 1), (p, 1, 1), 4, L, I.DIST_HALF_ZERO,
                              500 + j, nu, dt, nsteps, u0))
    return out


def standalone(gpu, w, nsteps, fuse=1):
    st = gpu.Stepper(n=w.n[0], p=w.p[0], order=w.order, L=w.L, nu=w.nu, dt=w.dt,
                     nsteps_max=w.nsteps, seed=w.seed, dist=w.dist)
    st.set_fuse(fuse)
    u = dev(w.u0)
    s = torch.empty_like(u)
    st.run(u, s, nsteps)
    return u, st


def test_batch_equals_standalone_and_oracle(gpu):
    wls = small_instances()
    nst = wls[0].nsteps
    refs = [standalone(gpu, w, nst)[0] for w in wls]
    _, st0 = standalone(gpu, wls[2], nst)
    o = oracle.run1d(wls[2].u0, wls[2].n[0], wls[2].p[0], 4, wls[2].L, wls[2].nu, wls[2].dt,
                     st0.delays(), nst)
    assert np.array_equal(refs[2].cpu().numpy(), o)
    b = gpu.Batch.from_workloads(wls)
    for s in (1, 2, 5, 8, 16, 32, 48, 64):
        if s > b.query()[2]:
            continue
        log("batch fuse", s)
        b.reset()
        b.set_fuse(s)
        us = [dev(w.u0) for w in wls]
        ss = [torch.empty_like(u) for u in us]
        b.run(us, ss, 50)
        b.run(us, ss, nst - 50)         # two calls: the shared step counter carries on
        for j in range(len(wls)):
            assert torch.equal(us[j], refs[j]), "instance %d fuse %d" % (j, s)


def test_batch_graph_replays(gpu):
    wls = small_instances(nsteps=64)
    b = gpu.Batch.from_workloads(wls)
    b.set_fuse(min(6, b.query()[2]))
    us = [dev(w.u0) for w in wls]
    ss = [torch.empty_like(u) for u in us]
    b.run(us, ss, 64, use_graph=False)
    eager = [u.clone() for u in us]
    for rep in range(3):
        b.reset()
        for u, w in zip(us, wls):
            u.copy_(dev(w.u0))
        torch.cuda.synchronize()
        b.run(us, ss, 64, use_graph=True)
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()      # eager work between replays
        for j in range(len(wls)):
            assert torch.equal(us[j], eager[j]), "replay %d instance %d" % (rep, j)
        del junk


def test_batch_rejects_unaligned_tiles(gpu):
    w = small_instances()[0]
    bad = dict(n=600, p=6, order=4, L=2, nu=0.01, dt=1e-5, nsteps_max=10)   # W = 100
    ok = dict(n=w.n[0], p=w.p[0], order=4, L=2, nu=0.01, dt=1e-5, nsteps_max=10)
    with pytest.raises(gpu.AtError) as e:
        gpu.Batch([ok, bad])
    assert e.value.status == gpu.AT_ERR_SHAPE


def test_batch_full_workload_sampled(gpu):
    """256 instances, N_j = 256*round(2^u/256), u ~ U[12,18], order 4,
    500 steps, fused + graph-replayed: sampled instances equal their standalone
    one-launch-per-step runs bit for bit, two small ones also the oracle."""
    wls = I.batch_instances()
    nst = wls[0].nsteps
    log("instances", len(wls), "points", sum(w.n[0] for w in wls))
    b = gpu.Batch.from_workloads(wls)
    us = [dev(w.u0) for w in wls]
    ss = [torch.empty_like(u) for u in us]
    order = np.argsort([w.n[0] for w in wls])
    sample = list(order[:3]) + list(order[-2:]) + [17, 101, 200]
    refs = {j: standalone(gpu, wls[j], nst)[0] for j in sample}
    # the autotuned pair (trials as long as the benchmark's), then the largest
    # steps per launch (the edge-history ring wraps many times per launch)
    s = b.autotune(us, 128)
    log("autotuned fuse", s, "variant", b.variant)
    for fuse in (s, b.query()[2]):
        b.reset()
        b.set_fuse(fuse)
        for u, w in zip(us, wls):
            u.copy_(dev(w.u0))
        b.run(us, ss, nst, use_graph=True)
        for j in sample:
            assert torch.equal(us[j], refs[j]), "instance %d fuse %d" % (j, fuse)
    for j in order[:2]:
        w = wls[j]
        _, st = standalone(gpu, w, 1)
        o = oracle.run1d(w.u0, w.n[0], w.p[0], 4, w.L, w.nu, w.dt, st.delays(), nst)
        got = us[j].cpu().numpy()
        assert np.max(np.abs(got - o)) <= 1e-12 * np.max(np.abs(o))
    for u in us:
        assert bool(torch.isfinite(u).all())


def test_batch_points_per_thread_variants_and_autotune(gpu):
    """Every points-per-thread variant of the batched kernel (16, 8, 4) at
    several steps per launch gives each instance's standalone bits; the
    autotuner picks a (variant, steps per launch) pair and keeps the bits."""
    wls = small_instances(nsteps=90)
    nst = wls[0].nsteps
    refs = [standalone(gpu, w, nst)[0] for w in wls]
    b = gpu.Batch.from_workloads(wls)
    for v in (1, 2, 3):
        b.set_variant(v)
        assert b.variant == v
        mf = b.query()[2]
        for s in sorted({1, 3, min(8, mf), mf}):
            b.reset()
            us = [dev(w.u0) for w in wls]
            ss = [torch.empty_like(u) for u in us]
            b.set_fuse(s)
            b.run(us, ss, nst, use_graph=(s == mf))
            torch.cuda.synchronize()
            for j, (u, r) in enumerate(zip(us, refs)):
                assert torch.equal(u, r), "variant %d, s %d, instance %d" % (v, s, j)
        log("  batch variant %d: steps per launch up to %d, bits equal" % (v, mf))
    b.reset()
    u0 = [dev(w.u0) for w in wls]
    s = b.autotune(u0, 30)
    log("  batch autotune: variant %d, steps per launch %d" % (b.variant, s))
    assert b.variant in (1, 2, 3) and 1 <= s <= b.query()[2]
    us = [u.clone() for u in u0]
    b.run(us, [torch.empty_like(u) for u in us], nst)
    torch.cuda.synchronize()
    assert all(torch.equal(u, r) for u, r in zip(us, refs))


def test_standalone_autotune_picks_points_per_thread(gpu):
    """The 1D autotuner searches points per thread (variants 1-3) together
    with steps per launch; the chosen pair gives the one-step bits."""
    w = small_instances(nsteps=200)[5]             # 8192 points, 32 tiles of 256
    ref, _ = standalone(gpu, w, 200)
    st = gpu.Stepper(n=w.n[0], p=w.p[0], order=w.order, L=w.L, nu=w.nu, dt=w.dt,
                     nsteps_max=w.nsteps, seed=w.seed, dist=w.dist)
    s = st.autotune(dev(w.u0), 60)
    log("  autotune: variant %d, steps per launch %d" % (st.variant, s))
    assert st.variant in (1, 2, 3) and st.query()[1] == s
    u = dev(w.u0)
    st.run(u, torch.empty_like(u), 200)
    assert torch.equal(u, ref)
