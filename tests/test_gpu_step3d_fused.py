"""GPU parity of the two-step 3D variants (15: 64 x 8 tiles, 16: 64 x 4 tiles;
levels n -> n+2 per launch) against the CPU oracle and against one launch per
step, through the C ABI.

Each launch recomputes level n+1 on a one-point rim around its tile as the
neighbouring block would (with that block's delays and AT halos, section 2
Eqs. (1)-(2)) and reads the ring's AT levels where the step-(n+1) delay is
positive; every point update is the one-step kernel's own sequence of
operations, so the bar is bit equality with the one-step run, and the oracle
tolerance (1e-12 normwise) is checked on top."""
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


CASES = [
    # name, n (x, y, z), p (x, y, z), L, dist, nu, nsteps, stale, alpha
    ("n64x32x24_p1x2x3_L3", (64, 32, 24), (1, 2, 3), 3, 0, 0.02, 31, False, ()),
    ("n128x64x40_p2x4x5_L3", (128, 64, 40), (2, 4, 5), 3, 0, 0.01, 24, False, ()),
    ("n128x24x20_p2x3x2_L2", (128, 24, 20), (2, 3, 2), 2, 1, 0.02, 27, False, ()),
    ("n64x16x16_p1x4x8_wz2", (64, 16, 16), (1, 4, 8), 3, 0, 0.02, 20, False, ()),
    ("n192x32x48_p3x2x4_L5", (192, 32, 48), (3, 2, 4), 5, 0, 0.01, 22, False, ()),
    ("n128x32x32_p1x2x2_wx128", (128, 32, 32), (1, 2, 2), 3, 0, 0.02, 19, False, ()),
    ("n64x32x32_p1x2x2_stale", (64, 32, 32), (1, 2, 2), 3, 0, 0.02, 21, True, ()),
    ("n64x24x24_p1x3x3_L0", (64, 24, 24), (1, 3, 3), 0, 0, 0.02, 18, False, ()),
    ("n64x16x24_p1x2x3_scal1", (64, 16, 24), (1, 2, 3), 3, 0, 0.02, 17, False, (0.01,)),
    ("n64x16x16_p1x2x2_scal2", (64, 16, 16), (1, 2, 2), 2, 0, 0.02, 15, False, (0.01, 0.03)),
]


def _field(n, nc, seed):
    u = I.u0_modes3d(n, 6, 3, seed)
    if nc > 3:
        u = np.concatenate([u] + [I.u0_modes3d(n, 5, 3, seed + 10 + j)[:1] for j in range(nc - 3)])
    return u


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_fused3d_parity(gpu, case):
    name, n, p, L, dist, nu, nst, stale, alpha = case
    log("3d two-step parity", name)
    nc = 3 + len(alpha)
    u0 = _field(n, nc, 5)
    dt = I.dt_rule(2 * math.pi / max(n), float(np.max(np.abs(u0[:3]))), nu)
    outs = {}
    k = None
    for var in (0, 15, 16):
        st = gpu.Stepper(dim=3, n=n, p=p, order=2, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=11,
                         dist=dist, halo_mode=1 if stale else 0, alpha=alpha)
        try:
            st.set_variant(var)
        except gpu.AtError as e:
            assert var == 16 or var == 15, var
            assert e.status == gpu.AT_ERR_ARG
            continue
        if var >= 15:
            assert st.query()[1] == 2
        u, s = dev(u0), torch.empty(u0.shape, dtype=torch.float64, device="cuda")
        st.run(u, s, nst)
        outs[var] = host(u)
        k = st.delays()
    assert any(v >= 15 for v in outs), "no two-step variant fits %s" % name
    ref = oracle.run3d(u0, n, p, L, nu, dt, k, nst, stale=stale, alpha=alpha)
    for var, got in outs.items():
        err = relerr(got, ref)
        log("  variant %d rel err %.3e bitwise %s" % (var, err, np.array_equal(got, ref)))
        assert err <= TOL, var
        assert np.array_equal(got, outs[0]), "variant %d differs from one step per launch" % var


def test_fused3d_mixed_launches_and_poison(gpu):
    """Runs split into pieces of odd length (two-step launches, then a single
    step), at_step in between, the poisoned ring (no read outside the levels
    the delay bound allows), and graph replay: all equal to the oracle."""
    n, p, L, nu, nst = (128, 32, 24), (2, 2, 3), 3, 0.02, 25
    u0 = _field(n, 3, 9)
    dt = I.dt_rule(2 * math.pi / 128, float(np.max(np.abs(u0))), nu)
    res = []
    for graph in (False, True):
        st = gpu.Stepper(dim=3, n=n, p=p, order=2, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=3)
        st.set_variant(15)
        st.set_debug(gpu.DEBUG_POISON_RING)
        st.set_graph(graph)
        u, s = dev(u0), torch.empty(u0.shape, dtype=torch.float64, device="cuda")
        st.run(u, s, 5)
        v = torch.empty_like(u)
        st.step(u, v)
        st.run(v, s, 7)
        st.run(v, s, nst - 13)
        res.append(host(v))
        k = st.delays()
    ref = oracle.run3d(u0, n, p, L, nu, dt, k, nst)
    for got in res:
        assert np.array_equal(got, ref)


def test_fused3d_full_size_first_steps(gpu):
    """512^3 x 3, 8^3 blocks of 64^3, L = 3: the two-step variants over the
    first 8 steps against the oracle (k reaches L = 3 from step 4 on), and
    all 200 steps equal to one launch per step bit for bit."""
    wl = I.wl_solenoidal_3d()
    log("3d two-step full size", wl.name)
    u0 = dev(wl.u0)
    outs = {}
    for var in (15, 16, 7):
        st = gpu.Stepper(dim=3, n=wl.n, p=wl.p, order=2, L=wl.L, nu=wl.nu, dt=wl.dt,
                         nsteps_max=wl.nsteps, seed=wl.seed, dist=wl.dist)
        st.set_variant(var)
        u, s = u0.clone(), torch.empty_like(u0)
        st.run(u, s, 8)
        outs[var] = host(u)
        k = st.delays()
        if var != 16:
            st.run(u, s, wl.nsteps - 8)
            outs[(var, "all")] = u.clone()
        del s, u
    ref = oracle.run3d(wl.u0, wl.n, wl.p, wl.L, wl.nu, wl.dt, k, 8)
    for var in (15, 16, 7):
        err = relerr(outs[var], ref)
        log("  variant %d, 8 steps: rel err %.3e bitwise %s" %
            (var, err, np.array_equal(outs[var], ref)))
        assert err <= TOL
    assert bool(torch.equal(outs[(15, "all")], outs[(7, "all")]))
