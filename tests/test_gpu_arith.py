"""Contracted arithmetic (arith = 1, 1D only): the stencil update and the AT
extrapolation use fused multiply-adds with dt*c1 and dt*nu*c2 folded into
two coefficients.  The result is no longer the oracle's bits, so the bar is
the floating-point tolerance, max|u_gpu - u_oracle| / max|u_oracle| <= 1e-12;
within the mode every launch form (one step per launch, fused steps, the
batched form) still gives identical bits, since all of them evaluate the
same expressions."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1911_05769_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-12


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relerr(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _inputs(N, nu, seed=3):
    u0 = I.u0_sines(N, seed) if N <= 1024 else I.u0_powerlaw(N, max(2, N // 16), seed)
    dt = I.dt_rule(2 * math.pi / N, float(np.max(np.abs(u0))), nu)
    return u0, dt


def run(gpu, u0, N, P, order, L, nu, dt, nst, fuse=1, arith=1, **kw):
    st = gpu.Stepper(n=N, p=P, order=order, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=7,
                     arith=arith, **kw)
    st.set_fuse(fuse)
    u, s = dev(u0), torch.empty(N, dtype=torch.float64, device="cuda")
    st.run(u, s, nst)
    return host(u), st


CASES = [
    # name, N, P, order, L, dist, nu, nsteps, extra
    ("sines_n1024_p8_o2_L2", 1024, 8, 2, 2, 0, 0.05, 1000, {}),
    ("powerlaw_n6000_p12_o4_L4", 6000, 12, 4, 4, 1, 1e-3, 400, {}),
    ("powerlaw_n8192_p16_o4_L3", 8192, 16, 4, 3, 0, 2e-3, 300, {}),
    ("single_tile_n512_o4", 512, 1, 4, 3, 1, 0.01, 200, {}),
    ("stale_n2048_p16_o2", 2048, 16, 2, 3, 0, 0.02, 300, {"halo_mode": 1}),
    ("linear_n2048_p8_o4", 2048, 8, 4, 2, 0, 0.02, 300, {"adv_mode": 1, "adv_speed": 0.8}),
    ("ragged_n12345_p5_o4", 12345, 5, 4, 3, 0, 0.01, 77, {}),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_contracted_parity_and_fused_bits(gpu, case):
    name, N, P, order, L, dist, nu, nst, extra = case
    log("contracted", name)
    u0, dt = _inputs(N, nu)
    if "adv_speed" in extra:
        dt = min(dt, 0.2 * (2 * math.pi / N) / extra["adv_speed"])
    plain, st = run(gpu, u0, N, P, order, L, nu, dt, nst, dist=dist, **extra)
    ref = oracle.run1d(u0, N, P, order, L, nu, dt, st.delays(), nst,
                       stale=extra.get("halo_mode") == 1, linear=extra.get("adv_mode") == 1,
                       adv_speed=extra.get("adv_speed", 0.0))
    err = relerr(plain, ref)
    log("  rel err %.3e" % err)
    assert err <= TOL
    exact, _ = run(gpu, u0, N, P, order, L, nu, dt, nst, arith=0, dist=dist, **extra)
    assert np.array_equal(exact, ref)                 # mode 0 untouched
    for s in (2, 3, 8, 16, 32, 48, 64):
        try:
            got, _ = run(gpu, u0, N, P, order, L, nu, dt, nst, fuse=s, dist=dist, **extra)
        except gpu.AtError as e:
            assert e.status == gpu.AT_ERR_ARG         # above this grid's limit
            continue
        assert np.array_equal(got, plain), "fuse %d differs" % s


def test_contracted_full_size(gpu):
    """N = 2^24, P = 4096, order 4, L = 4 in the contracted mode: 200 autotuned
    steps against the oracle, then all 2000 steps fused against one launch
    per step, bit for bit."""
    wl = I.wl_powerlaw_1d()
    N, P = wl.n[0], wl.p[0]
    log("contracted full size", wl.name)
    st = gpu.Stepper(n=N, p=P, order=wl.order, L=wl.L, nu=wl.nu, dt=wl.dt, nsteps_max=wl.nsteps,
                     seed=wl.seed, dist=wl.dist, arith=1)
    u0 = dev(wl.u0)
    s = st.autotune(u0, 40)
    log("  autotuned fuse", s)
    u, scr = u0.clone(), torch.empty_like(u0)
    st.run(u, scr, 200)
    ref = oracle.run1d(wl.u0, N, P, wl.order, wl.L, wl.nu, wl.dt, st.delays(), 200)
    err = relerr(host(u), ref)
    log("  200 steps rel err %.3e" % err)
    assert err <= TOL
    st.run(u, scr, wl.nsteps - 200)
    st2 = gpu.Stepper(n=N, p=P, order=wl.order, L=wl.L, nu=wl.nu, dt=wl.dt,
                      nsteps_max=wl.nsteps, seed=wl.seed, dist=wl.dist, arith=1)
    st2.set_fuse(1)
    v = u0.clone()
    st2.run(v, scr, wl.nsteps)
    assert torch.equal(u, v)
    assert bool(torch.isfinite(u).all())


def test_contracted_batch_equals_standalone(gpu):
    g = np.random.default_rng(9)
    wls = []
    for j, (n, p) in enumerate([(1024, 8), (4096, 16), (768, 3), (8192, 32), (256, 1)]):
        nu = float(g.uniform(1e-3, 5e-2))
        u0 = I.u0_powerlaw(n, n // 16, 40 + j)
        dt = I.dt_rule(2 * math.pi / n, float(np.max(np.abs(u0))), nu)
        wls.append(I.Workload("c%d" % j, 1, (n, 1, 1), (p, 1, 1), 4, 3, I.DIST_HALF_ZERO,
                              60 + j, nu, dt, 90, u0))
    b = gpu.Batch.from_workloads(wls, arith=1)
    b.set_fuse(min(8, b.query()[2]))
    us = [dev(w.u0) for w in wls]
    ss = [torch.empty_like(u) for u in us]
    b.run(us, ss, 90, use_graph=True)
    for j, w in enumerate(wls):
        st = gpu.Stepper(n=w.n[0], p=w.p[0], order=4, L=w.L, nu=w.nu, dt=w.dt, nsteps_max=90,
                         seed=w.seed, dist=w.dist, arith=1)
        u = dev(w.u0)
        st.run(u, torch.empty_like(u), 90)
        assert torch.equal(us[j], u), "instance %d" % j
        ref = oracle.run1d(w.u0, w.n[0], w.p[0], 4, w.L, w.nu, w.dt, st.delays(), 90)
        assert relerr(host(u), ref) <= TOL


def test_contracted_adjoint_close(gpu):
    """Record mode and the adjoint run on top of contracted forward steps: the
    gradient (dJ/du0 normwise, dJ/dnu relative) must stay within the 1e-12
    tolerance of the oracle's adjoint of the exact-order scheme, like the
    contracted forward field itself."""
    N, P, order, L, nu, nst = 2048, 8, 4, 2, 5e-3, 200
    u0, dt = _inputs(N, nu, seed=8)
    tgt = I.u0_powerlaw(N, N // 16, 9)
    st = gpu.Stepper(n=N, p=P, order=order, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=5,
                     record=True, ckpt_every=50, arith=1)
    u, s = dev(u0), torch.empty(N, dtype=torch.float64, device="cuda")
    st.run(u, s, nst)
    lam = torch.empty_like(u)
    st.loss(u, dev(tgt), lam)
    g_u0, g_nu = st.adjoint(lam)
    k = st.delays()
    uT = oracle.run1d(u0, N, P, order, L, nu, dt, k, nst)
    assert relerr(host(u), uT) <= TOL
    _, lamT = oracle.loss(uT, tgt)
    lam0, gnu_ref = oracle.adjoint1d(u0, lamT, N, P, order, L, nu, dt, k, nst)
    e = relerr(host(g_u0), lam0)
    en = abs(float(host(g_nu)[0]) - gnu_ref) / abs(gnu_ref)
    log("  contracted adjoint: grad u0 rel %.3e, grad nu rel %.3e" % (e, en))
    assert e <= TOL
    assert en <= TOL
