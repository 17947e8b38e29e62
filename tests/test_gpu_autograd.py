"""The torch.autograd.Function over the AT stepper (AtBurgers, AtMisfit).

J = 0.5 ||u(T) - u*||^2 is formed by AtMisfit from AtBurgers' final field;
J.backward() runs the library's discrete adjoint.  Checked:
  * u0.grad and nu.grad against the CPU oracle's brute-force adjoint
    (normwise relative <= 1e-12; dJ/dnu relative <= 1e-12), the forward field
    bit for bit and J within 1e-14 relative;
  * the adjoint workload's grid and launch configuration (N = 2^20,
    P = 1024, order 2, L = 3, checkpoints every 100 steps, fused forward and
    reverse launches) against the oracle over its first 300 steps;
  * the full adjoint workload (4000 steps) against central finite
    differences (h = 1e-6) on 16 seeded directions and on nu;
  * use from a side stream (every launch on the stream current at apply
    time), with the same bits as on the default stream.
Gradients are those of the discrete map with dt held fixed (the paper's
scheme, section 2 Eqs. (1)-(2) and section 3.2, differentiated)."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_1911_05769_amd import autograd as AG
from paper_1911_05769_amd import inputs as I

pytestmark = pytest.mark.gpu
TOL = 1e-12


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relerr(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def grads(u0_np, tgt_np, nu, spec, nu_on_gpu=False):
    """(uT, J, dJ/du0, dJ/dnu) through AtBurgers -> AtMisfit -> backward."""
    u0 = dev(u0_np).requires_grad_()
    nut = torch.tensor(nu, dtype=torch.float64, device="cuda" if nu_on_gpu else "cpu",
                       requires_grad=True)
    uT = AG.AtBurgers.apply(u0, nut, spec)
    J = AG.AtMisfit.apply(uT, dev(tgt_np))
    J.backward()
    assert nut.grad.device == nut.device and nut.grad.shape == nut.shape
    return host(uT), float(host(J)), host(u0.grad), float(nut.grad.detach().cpu())


def oracle_grads(u0, tgt, spec, nu):
    m = oracle.levels_for_order(spec.order)
    k = oracle.delays(spec.nsteps, 2 * spec.p, spec.L, m, spec.dist, spec.seed)
    uT = oracle.run1d(u0, spec.n, spec.p, spec.order, spec.L, nu, spec.dt, k, spec.nsteps)
    J, lamT = oracle.loss(uT, tgt)
    lam0, gnu = oracle.adjoint1d(u0, lamT, spec.n, spec.p, spec.order, spec.L, nu, spec.dt, k,
                                 spec.nsteps)
    return uT, J, lam0, gnu


CASES = [
    # name, N, P, order, L, dist, nu, nsteps, C
    ("o2_n2048_p16_L3_C50", 2048, 16, 2, 3, 0, 0.02, 300, 50),
    ("o4_n1536_p12_L4_C64", 1536, 12, 4, 4, 1, 0.01, 200, 64),
    ("o2_n4096_p512_w8_C37", 4096, 512, 2, 3, 1, 0.02, 150, 37),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_autograd_against_oracle_adjoint(gpu, case):
    name, N, P, order, L, dist, nu, nst, C = case
    log("autograd", name)
    u0 = I.u0_powerlaw(N, N // 16, 31)
    tgt = I.u0_powerlaw(N, 16, 99) * 0.5
    dt = I.dt_rule(2 * math.pi / N, float(np.max(np.abs(u0))), nu)
    spec = AG.StepSpec(n=N, p=P, order=order, L=L, dt=dt, nsteps=nst, ckpt_every=C, seed=7,
                       dist=dist)
    uT, J, g, gnu = grads(u0, tgt, nu, spec, nu_on_gpu=(order == 4))
    uT_r, J_r, g_r, gnu_r = oracle_grads(u0, tgt, spec, nu)
    e, en = relerr(g, g_r), abs(gnu - gnu_r) / abs(gnu_r)
    log("  forward bitwise %s, J rel %.2e, grad u0 rel %.3e, grad nu rel %.3e" %
        (np.array_equal(uT, uT_r), abs(J - J_r) / J_r, e, en))
    assert np.array_equal(uT, uT_r)
    assert abs(J - J_r) <= 1e-14 * J_r
    assert e <= TOL
    assert en <= TOL


def test_autograd_full_grid_first_steps_against_oracle(gpu):
    """The adjoint workload's grid and launch configuration over its first 300
    steps (three checkpoint segments of 100, fused forward launches, fused
    reverse launches of up to 64 steps), against the oracle's adjoint."""
    wl = I.wl_adjoint_1d()
    N, P, C, nst = wl.n[0], wl.p[0], wl.extra["ckpt"], 300
    log("autograd full grid", wl.name, "first", nst, "steps")
    spec = AG.StepSpec(n=N, p=P, order=2, L=wl.L, dt=wl.dt, nsteps=nst, ckpt_every=C,
                       seed=wl.seed, dist=wl.dist)
    tgt = I.u0_powerlaw(N, N // 16, wl.seed + 5)
    uT, J, g, gnu = grads(wl.u0, tgt, wl.nu, spec)
    uT_r, J_r, g_r, gnu_r = oracle_grads(wl.u0, tgt, spec, wl.nu)
    e, en = relerr(g, g_r), abs(gnu - gnu_r) / abs(gnu_r)
    log("  forward bitwise %s, grad u0 rel %.3e, grad nu rel %.3e" %
        (np.array_equal(uT, uT_r), e, en))
    assert np.array_equal(uT, uT_r)
    assert abs(J - J_r) <= 1e-14 * J_r
    assert e <= TOL
    assert en <= TOL


def test_autograd_full_size_fd(gpu):
    """The full adjoint workload (N = 2^20, P = 1024, order 2, L = 3, 4000
    steps, checkpoints every 100; the target is u0 run at nu = 3e-3): the
    autograd gradient against central finite differences, h = 1e-6, on 16
    seeded N(0,1) directions of u0 and on nu."""
    wl = I.wl_adjoint_1d()
    N, P, nst, C = wl.n[0], wl.p[0], wl.nsteps, wl.extra["ckpt"]
    log("autograd full size fd", wl.name)
    from paper_1911_05769_amd import at
    scr = torch.empty(N, dtype=torch.float64, device="cuda")

    def run(nu, u_init):
        st = at.Stepper(n=N, p=P, order=2, L=wl.L, nu=nu, dt=wl.dt, nsteps_max=nst,
                        seed=wl.seed, dist=wl.dist, fuse_steps=32)
        u = u_init.clone()
        st.run(u, scr, nst)
        return st, u

    _, target = run(wl.extra["nu_target"], dev(wl.u0))
    spec = AG.StepSpec(n=N, p=P, order=2, L=wl.L, dt=wl.dt, nsteps=nst, ckpt_every=C,
                       seed=wl.seed, dist=wl.dist)
    _, J0, g, gnu = grads(wl.u0, host(target), wl.nu, spec)
    h = 1e-6

    def J(nu, u_init):
        st, u = run(nu, u_init)
        return float(host(st.loss(u, target))[0])

    u0 = dev(wl.u0)
    worst = 0.0
    for d in I.fd_directions(N, 16, wl.seed + 1):
        dd = dev(d)
        fd = (J(wl.nu, u0 + h * dd) - J(wl.nu, u0 - h * dd)) / (2 * h)
        worst = max(worst, abs(fd - float(np.dot(g, d))) / abs(fd))
    fdn = (J(wl.nu + h, u0) - J(wl.nu - h, u0)) / (2 * h)
    en = abs(fdn - gnu) / abs(fdn)
    log("  J %.4e, worst direction rel %.3e, nu rel %.3e" % (J0, worst, en))
    assert worst <= 1e-6
    assert en <= 1e-6


def test_autograd_on_side_stream(gpu):
    """Applied under a side stream, every launch (forward, loss, adjoint) goes
    to that stream: the same bits as on the default stream, and the loss
    reduction runs on a context bound to that stream."""
    N, P, order, L, nu, nst, C = 2048, 16, 2, 3, 0.02, 200, 50
    u0 = I.u0_powerlaw(N, N // 16, 41)
    tgt = I.u0_powerlaw(N, 16, 42)
    dt = I.dt_rule(2 * math.pi / N, float(np.max(np.abs(u0))), nu)
    spec = AG.StepSpec(n=N, p=P, order=order, L=L, dt=dt, nsteps=nst, ckpt_every=C, seed=3)
    ref = grads(u0, tgt, nu, spec)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        got = grads(u0, tgt, nu, spec)
        red = AG._reducer(N, torch.device("cuda"))
        assert red.stream.cuda_stream == side.cuda_stream
    torch.cuda.current_stream().wait_stream(side)
    assert np.array_equal(got[0], ref[0]) and got[1] == ref[1]
    assert np.array_equal(got[2], ref[2]) and got[3] == ref[3]
