"""GPU parity of the whole-grid single-workgroup 1D variant (at_set_variant 4)
against the CPU oracle and against the other launch forms, through the C ABI.

The variant holds the whole periodic grid in one workgroup, so the neighbour
exchange wraps around and one launch advances a whole run.  Every update is
the same sequence of operations as in the other kernels (section 3.2 stencil,
section 2 Eqs. (1)-(2) halos), so the bar is bit equality with the oracle and
with one launch per step."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1911_05769_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-12
WHOLE = 4


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _inputs(N, nu, seed=3):
    u0 = I.u0_sines(N, seed) if N <= 1024 else I.u0_powerlaw(N, max(2, N // 16), seed)
    return u0, I.dt_rule(2 * math.pi / N, float(np.max(np.abs(u0))), nu)


CASES = [
    # name, N, P, order, L, dist, nu, nsteps, extra
    ("c1_n1024_p8_o2_L2", 1024, 8, 2, 2, 0, 0.05, 1000, {}),
    ("single_tile_n512_o4", 512, 1, 4, 3, 1, 0.01, 300, {}),
    ("n4096_p16_o4_L4_ppt16", 4096, 16, 4, 4, 1, 1e-3, 400, {}),
    ("n2048_p64_o2_ppt8", 2048, 64, 2, 3, 0, 0.02, 250, {}),
    ("n96_p3_o4_tiny", 96, 3, 4, 2, 1, 0.02, 120, {}),
    ("n1024_p256_w4_o2", 1024, 256, 2, 3, 0, 0.02, 150, {}),
    ("stale_n1024_p8", 1024, 8, 2, 3, 0, 0.02, 200, {"halo_mode": 1}),
    ("linear_n2048_p8_o4", 2048, 8, 4, 2, 0, 0.02, 200, {"adv_mode": 1, "adv_speed": 0.8}),
    ("max_delay_n1024_p8_o2_L15", 1024, 8, 2, 15, 1, 0.02, 200, {}),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_whole_grid_parity(gpu, case):
    name, N, P, order, L, dist, nu, nst, extra = case
    log("whole grid", name)
    u0, dt = _inputs(N, nu)
    if "adv_speed" in extra:
        dt = min(dt, 0.2 * (2 * math.pi / N) / extra["adv_speed"])
    st = gpu.Stepper(n=N, p=P, order=order, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=7,
                     dist=dist, **extra)
    st.set_variant(WHOLE)
    assert st.variant == WHOLE and st.query()[1] == nst
    u, s = dev(u0), torch.empty(N, dtype=torch.float64, device="cuda")
    # uneven pieces: launches start at many different steps
    done = 0
    for piece in (1, 2, 37, nst):
        m = min(piece, nst - done)
        if m > 0:
            st.run(u, s, m)
            done += m
    got = host(u)
    ref = oracle.run1d(u0, N, P, order, L, nu, dt, st.delays(), nst,
                       stale=extra.get("halo_mode") == 1, linear=extra.get("adv_mode") == 1,
                       adv_speed=extra.get("adv_speed", 0.0))
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    log("  rel err %.3e bitwise %s" % (err, np.array_equal(got, ref)))
    assert err <= TOL
    assert np.array_equal(got, ref)


def test_whole_grid_mixed_with_other_forms(gpu):
    """Whole-grid launches, single steps (at_step) and fused launches of the
    regular kernels in one run, with ring poisoning and graph replay: the
    ring the whole-grid kernel leaves is the one the other forms read."""
    N, P, order, L, nu, nst = 1024, 8, 4, 4, 0.02, 300
    u0, dt = _inputs(N, nu, seed=5)
    ref = None
    for graph in (False, True):
        st = gpu.Stepper(n=N, p=P, order=order, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=9,
                         dist=1)
        st.set_debug(gpu.DEBUG_POISON_RING)
        st.set_graph(graph)
        u, s = dev(u0), torch.empty(N, dtype=torch.float64, device="cuda")
        st.set_variant(WHOLE)
        st.run(u, s, 57)
        v = torch.empty_like(u)
        st.step(u, v)                                 # one step, whole-grid kernel
        st.set_variant(0)
        st.set_fuse(13)
        st.run(v, s, 40)                              # regular fused launches
        st.step(v, u)
        st.set_variant(WHOLE)
        st.run(u, s, nst - 99)
        got = host(u)
        if ref is None:
            ref = oracle.run1d(u0, N, P, order, L, nu, dt, st.delays(), nst)
        assert np.array_equal(got, ref), "graph %s" % graph


def test_whole_grid_contracted_equals_fused_contracted(gpu):
    """Contracted arithmetic: the whole-grid kernel gives the bits of the
    regular fused kernels in the same mode, within 1e-12 of the oracle."""
    N, P, order, L, nu, nst = 2048, 16, 4, 3, 0.01, 300
    u0, dt = _inputs(N, nu, seed=6)
    outs = []
    for v in (WHOLE, 0):
        st = gpu.Stepper(n=N, p=P, order=order, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=4,
                         dist=1, arith=1)
        st.set_variant(v)
        if v == 0:
            st.set_fuse(16)
        u, s = dev(u0), torch.empty(N, dtype=torch.float64, device="cuda")
        st.run(u, s, nst)
        outs.append(host(u))
        k = st.delays()
    assert np.array_equal(outs[0], outs[1])
    ref = oracle.run1d(u0, N, P, order, L, nu, dt, k, nst)
    assert float(np.max(np.abs(outs[0] - ref)) / np.max(np.abs(ref))) <= TOL


def test_whole_grid_record_mode_adjoint(gpu):
    """Record mode: the whole-grid forward writes the full edge tape, so the
    adjoint (rebuilt with the regular kernels) equals that of a regular
    forward run bit for bit, and the oracle's within 1e-12."""
    N, P, order, L, nu, nst, C = 2048, 16, 2, 3, 0.02, 300, 50
    u0, dt = _inputs(N, nu, seed=8)
    tgt = I.u0_powerlaw(N, 16, 9)
    res = []
    for v in (WHOLE, 0):
        st = gpu.Stepper(n=N, p=P, order=order, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=5,
                         record=True, ckpt_every=C)
        st.set_variant(v)
        u, s = dev(u0), torch.empty(N, dtype=torch.float64, device="cuda")
        st.run(u, s, nst)
        lam = torch.empty_like(u)
        st.loss(u, dev(tgt), lam)
        g, gnu = st.adjoint(lam)
        res.append((host(u), host(g), host(gnu)))
        k = st.delays()
    assert all(np.array_equal(a, b) for a, b in zip(res[0], res[1]))
    uT = oracle.run1d(u0, N, P, order, L, nu, dt, k, nst)
    assert np.array_equal(res[0][0], uT)
    _, lamT = oracle.loss(uT, tgt)
    lam0, gnu_ref = oracle.adjoint1d(u0, lamT, N, P, order, L, nu, dt, k, nst)
    assert float(np.max(np.abs(res[0][1] - lam0)) / np.max(np.abs(lam0))) <= TOL
    assert abs(float(res[0][2][0]) - gnu_ref) <= TOL * abs(gnu_ref)


def test_whole_grid_autotune_and_refusals(gpu):
    """The autotuner may choose the whole-grid variant for the small C1 grid
    (any choice gives the oracle's bits); grids that do not fit one workgroup
    refuse it."""
    wl = I.wl_sines_1d()
    N, P = wl.n[0], wl.p[0]
    st = gpu.Stepper(n=N, p=P, order=2, L=wl.L, nu=wl.nu, dt=wl.dt, nsteps_max=wl.nsteps,
                     seed=wl.seed, dist=wl.dist)
    u0 = dev(wl.u0)
    s = st.autotune(u0, 200)
    log("  C1 autotune: variant %d, steps per launch %d" % (st.variant, s))
    u, scr = u0.clone(), torch.empty_like(u0)
    st.run(u, scr, wl.nsteps)
    ref = oracle.run1d(wl.u0, N, P, 2, wl.L, wl.nu, wl.dt, st.delays(), wl.nsteps)
    assert np.array_equal(host(u), ref)
    for n, p in ((1 << 14, 8), (1000, 8), (1 << 12, 2048)):
        big = gpu.Stepper(n=n, p=p, order=2, L=2, nu=0.01, dt=1e-6, nsteps_max=4)
        with pytest.raises(gpu.AtError) as e:
            big.set_variant(WHOLE)
        assert e.value.status == gpu.AT_ERR_ARG
