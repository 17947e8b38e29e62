"""The paper's accuracy study run on the GPU path (section 3.2, Figure 2;
Eq. (3)), through the C ABI, with the production kernels (fused launches):

* convergence against closed-form solutions (Cole-Hopf Burgers and linear
  advection-diffusion, orders 2 and 4): the synchronous scheme and the AT
  scheme converge at order 2 (dt ~ dx^2 forward Euler dominates), the
  standard stencil fed with delayed halo values (the stale mode) drops to
  order 1 -- Figure 2's three curves;
* the error law of Eq. (3), <E> ~ (P/N) dx^2 (<k^2> + <k>): the AT-minus-
  synchronous difference grows linearly in P at fixed N, is proportional to
  <k^2> + <k> at fixed N and P, and falls at order 3 in N at fixed P.

Grids go larger than the oracle's pins of the same laws (N up to 2048,
P up to 64).  Each table is logged; one GPU run per family is also checked
against the oracle bit for bit."""
import math
import sys

import numpy as np
import pytest
import torch

import oracle
from exact import AdvDiff1D, ColeHopf1D

pytestmark = pytest.mark.gpu


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_final(gpu, u0, N, P, order, L, nu, dt, nst, mode, linear=False, c=0.0, seed=11,
              fuse=8):
    m = 2 if order == 2 else 3
    kw = dict(n=N, p=P, order=order, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=seed, dist=0,
              halo_mode=1 if mode == "stale" else 0)
    if linear:
        kw.update(adv_mode=1, adv_speed=c)
    if mode == "sync":
        kw["delays"] = np.zeros((nst, 2 * P), np.int8)
    st = gpu.Stepper(**kw)
    while True:                                       # fused launches, within this grid's limit
        try:
            st.set_fuse(fuse)
            break
        except gpu.AtError:
            fuse -= 1
    u = torch.from_numpy(np.ascontiguousarray(u0)).cuda()
    s = torch.empty_like(u)
    st.run(u, s, nst)
    torch.cuda.synchronize()
    return u.cpu().numpy(), st.delays(), m


def _setup(N, nu, T):
    dx = 2 * np.pi / N
    dt = 0.1 * dx * dx / nu
    nst = int(round(T / dt))
    return dx, dt, nst, np.arange(N) * dx


@pytest.mark.parametrize("prob", ["burgers", "advdiff"])
@pytest.mark.parametrize("order", [2, 4])
def test_convergence_orders_figure2_on_gpu(gpu, prob, order):
    nu, T, P, L = 0.1, 0.25, 8, 3
    Ns = (64, 128, 256, 512, 1024)
    ex = ColeHopf1D(nu) if prob == "burgers" else AdvDiff1D(nu, 1.0)
    lin, c = (prob == "advdiff"), (1.0 if prob == "advdiff" else 0.0)
    errs = {}
    for mode in ("sync", "at", "stale"):
        errs[mode] = []
        for N in Ns:
            dx, dt, nst, x = _setup(N, nu, T)
            uT, k, _ = gpu_final(gpu, ex.u(x, 0.0), N, P, order, L, nu, dt, nst, mode,
                                 linear=lin, c=c)
            if N == 128:                      # the same run on the oracle: same bits
                ref = oracle.run1d(ex.u(x, 0.0), N, P, order, L, nu, dt, k, nst,
                                   stale=(mode == "stale"), linear=lin, adv_speed=c)
                assert np.array_equal(uT, ref), (mode, N)
            e = uT - ex.u(x, nst * dt)
            errs[mode].append(float(np.sqrt(np.mean(e * e))))
    orders = {mode: [math.log2(v[i] / v[i + 1]) for i in range(len(v) - 1)]
              for mode, v in errs.items()}
    log("convergence %s order %d (N = %s)" % (prob, order, Ns))
    for mode in ("sync", "at", "stale"):
        log("  %-5s rms err %s  orders %s" % (mode, " ".join("%.3e" % v for v in errs[mode]),
                                              " ".join("%.2f" % o for o in orders[mode])))
    assert abs(orders["sync"][-1] - 2.0) < 0.1
    assert abs(orders["at"][-1] - 2.0) < 0.15
    assert abs(orders["stale"][-1] - 1.0) < 0.2


def _at_minus_sync(gpu, N, P=8, L=3, order=2, nu=0.1, T=0.25, seed=11):
    dx, dt, nst, x = _setup(N, nu, T)
    u0 = ColeHopf1D(nu).u(x, 0.0)
    a, k, m = gpu_final(gpu, u0, N, P, order, L, nu, dt, nst, "at", seed=seed)
    s, _, _ = gpu_final(gpu, u0, N, P, order, L, nu, dt, nst, "sync", seed=seed)
    kk = k[m + L:].astype(np.float64)
    return float(np.mean(np.abs(a - s))), float(kk.mean()), float((kk * kk).mean())


def test_error_law_eq3_on_gpu(gpu):
    Ps = (4, 8, 16, 32, 64)
    eP = [_at_minus_sync(gpu, 1024, P=P)[0] for P in Ps]
    sP = [math.log2(eP[i + 1] / eP[i]) for i in range(len(Ps) - 1)]
    log("error law: N = 1024, L = 3: <|AT - sync|> vs P %s: %s  slopes %s" % (
        Ps, " ".join("%.3e" % v for v in eP), " ".join("%.2f" % v for v in sP)))
    Ls = (1, 2, 4, 8)
    rows = [_at_minus_sync(gpu, 1024, P=16, L=L) for L in Ls]
    ratios = [e / (k1 + k2) for e, k1, k2 in rows]
    log("error law: N = 1024, P = 16: L %s, <k^2>+<k> %s, E/(<k^2>+<k>) %s" % (
        Ls, " ".join("%.3f" % (k1 + k2) for _, k1, k2 in rows),
        " ".join("%.3e" % r for r in ratios)))
    Ns = (128, 256, 512, 1024, 2048)
    eN = [_at_minus_sync(gpu, N, P=8)[0] for N in Ns]
    sN = [math.log2(eN[i] / eN[i + 1]) for i in range(len(Ns) - 1)]
    log("error law: P = 8, L = 3: <|AT - sync|> vs N %s: %s  orders %s" % (
        Ns, " ".join("%.3e" % v for v in eN), " ".join("%.2f" % v for v in sN)))
    assert all(0.7 < v < 1.3 for v in sP), sP
    assert max(ratios) / min(ratios) < 1.2, ratios
    assert abs(sN[-1] - 3.0) < 0.3, sN
