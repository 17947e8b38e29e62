"""Graph replay of at_run, the ring-poisoning debug mode and snapshot/restore.

* Graph replay (at_set_graph): the captured launch sequence of a run gives the
  eager run's bits on every replay, with eager work and synchronisations of
  the program's own between replays; also in record mode, where the adjoint
  then matches the eager one.
* AT_DEBUG_POISON_RING: every ring slot outside the window of levels that the
  delay bound allows (section 2: levels n-k, ..., n-k-m+1 with k <= L) is
  NaN after each launch; the runs still equal the oracle bit for bit, so no
  kernel reads outside that window.
* at_restore of a buffer this context wrote takes the step from the host;
  a buffer from another context is read to find its step."""
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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _sines(N, nu, seed=3):
    u0 = I.u0_sines(N, seed)
    return u0, I.dt_rule(2 * math.pi / N, float(np.max(np.abs(u0))), nu)


@pytest.mark.parametrize("N,P,order,L,fuse,nst", [(1024, 8, 2, 2, 1, 1000),
                                                   (4096, 16, 4, 4, 8, 301),
                                                   (1000, 8, 4, 2, 1, 200)])
def test_graph_replay_equals_eager(gpu, N, P, order, L, fuse, nst):
    log("graph 1d", N, P, order, L, fuse, nst)
    nu = 0.05
    u0, dt = _sines(N, nu)
    eager = gpu.Stepper(n=N, p=P, order=order, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=9,
                        fuse_steps=fuse)
    u, s = dev(u0), torch.empty(N, dtype=torch.float64, device="cuda")
    eager.run(u, s, nst)
    ref = host(u)
    assert np.array_equal(ref, oracle.run1d(u0, N, P, order, L, nu, dt, eager.delays(), nst))
    st = gpu.Stepper(n=N, p=P, order=order, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=9,
                     fuse_steps=fuse)
    st.set_graph(True)
    g = torch.empty(N, dtype=torch.float64, device="cuda")
    snap = st.snapshot(dev(u0))
    junk = torch.ones(1 << 20, dtype=torch.float64, device="cuda")
    for rep in range(4):                       # capture, then three replays
        st.restore(snap, g)
        st.run(g, s, nst)
        assert st.n == nst
        got = host(g)
        assert np.array_equal(got, ref), "replay %d" % rep
        junk.mul_(1.0001)                      # eager work between replays
        torch.cuda.synchronize()
    # split runs (two graphs in turn) give the same bits
    st.restore(snap, g)
    st.run(g, s, nst // 2)
    st.run(g, s, nst - nst // 2)
    assert np.array_equal(host(g), ref)


def test_graph_replay_3d_and_record_mode(gpu):
    n, p, L, nu, nst = (48, 32, 24), (3, 2, 2), 3, 0.02, 25
    u0 = I.u0_modes3d(n, 6, 3, 4)
    dt = I.dt_rule(2 * math.pi / 48, float(np.max(np.abs(u0))), nu)
    outs = []
    for graph in (False, True, True):
        st = gpu.Stepper(dim=3, n=n, p=p, order=2, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=2)
        st.set_graph(graph)
        u, s = dev(u0), torch.empty(u0.shape, dtype=torch.float64, device="cuda")
        st.run(u, s, nst)
        outs.append(host(u))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    # record mode: graph-replayed forward, then the adjoint, equal to eager
    N, P, order, L1, nst1, C = 2048, 16, 2, 3, 200, 50
    u0, dt = _sines(N, 0.02)
    tgt = I.u0_powerlaw(N, 16, 5)
    res = []
    for graph in (False, True):
        st = gpu.Stepper(n=N, p=P, order=order, L=L1, nu=0.02, dt=dt, nsteps_max=nst1, seed=4,
                         record=True, ckpt_every=C, fuse_steps=16)
        st.set_graph(graph)
        u, s = dev(u0), torch.empty(N, dtype=torch.float64, device="cuda")
        st.run(u, s, nst1)
        lam = torch.empty_like(u)
        st.loss(u, dev(tgt), lam)
        gu, gnu = st.adjoint(lam)
        res.append((host(u), host(gu), host(gnu)))
    assert all(np.array_equal(a, b) for a, b in zip(res[0], res[1]))


POISON_1D = [
    # N, P, order, L, dist, fuse, nsteps
    (1024, 8, 2, 2, 0, 1, 300),
    (1024, 8, 2, 2, 0, 7, 300),
    (4096, 16, 4, 4, 1, 1, 200),
    (4096, 16, 4, 4, 1, 13, 200),
    (1000, 8, 4, 3, 0, 1, 150),        # tiles of 125 points: the general kernel
    (3000, 1, 2, 5, 0, 4, 120),
]


@pytest.mark.parametrize("case", POISON_1D, ids=["-".join(map(str, c)) for c in POISON_1D])
def test_poisoned_ring_same_bits_1d(gpu, case):
    N, P, order, L, dist, fuse, nst = case
    log("poison 1d", case)
    nu = 0.03
    u0, dt = _sines(N, nu, seed=6)
    st = gpu.Stepper(n=N, p=P, order=order, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=12,
                     dist=dist, fuse_steps=fuse)
    st.set_debug(gpu.DEBUG_POISON_RING)
    u, s = dev(u0), torch.empty(N, dtype=torch.float64, device="cuda")
    # in pieces of uneven length, so launches start at many different steps
    done = 0
    for piece in (1, 2, 37, nst):
        m = min(piece, nst - done)
        if m > 0:
            st.run(u, s, m)
            done += m
    got = host(u)
    ref = oracle.run1d(u0, N, P, order, L, nu, dt, st.delays(), nst)
    assert np.array_equal(got, ref)
    # the poison is in place: every slot outside the live window holds NaN
    n_, _, R = st.query()
    h, m_lev = order // 2, oracle.levels_for_order(order)
    lev = P * 2 * h
    buf = host(st.snapshot(u)).view(np.float64)
    off = (N * 8 + 255) // 256 * 256 // 8
    ring = buf[off:off + R * lev].reshape(R, lev)
    live = {q % R for q in range(max(0, nst - (L + m_lev - 1)), nst)}
    for slot in range(R):
        assert np.isnan(ring[slot]).all() == (slot not in live), slot


def test_poisoned_ring_same_bits_3d(gpu):
    n, p, L, nu, nst = (64, 48, 40), (1, 3, 2), 3, 0.02, 23
    u0 = I.u0_modes3d(n, 6, 3, 7)
    dt = I.dt_rule(2 * math.pi / 64, float(np.max(np.abs(u0))), nu)
    outs = {}
    for var in (0, 6, 9):
        st = gpu.Stepper(dim=3, n=n, p=p, order=2, L=L, nu=nu, dt=dt, nsteps_max=nst, seed=8)
        try:
            st.set_variant(var)
        except gpu.AtError:
            continue
        st.set_debug(gpu.DEBUG_POISON_RING)
        u, s = dev(u0), torch.empty(u0.shape, dtype=torch.float64, device="cuda")
        st.run(u, s, 5)
        for _ in range(nst - 5):
            v = torch.empty_like(u)
            st.step(u, v)
            u = v
        outs[var] = host(u)
        k = st.delays()
    ref = oracle.run3d(u0, n, p, L, nu, dt, k, nst)
    assert len(outs) >= 2
    for var, got in outs.items():
        assert np.array_equal(got, ref), "variant %d" % var


def test_poison_refused_in_record_mode(gpu):
    st = gpu.Stepper(n=1024, p=8, order=2, L=2, nu=0.05, dt=1e-5, nsteps_max=10, record=True,
                     ckpt_every=5)
    with pytest.raises(gpu.AtError) as e:
        st.set_debug(gpu.DEBUG_POISON_RING)
    assert e.value.status == gpu.AT_ERR_STATE
    with pytest.raises(gpu.AtError):
        st.set_debug(8)


def test_restore_from_another_contexts_snapshot(gpu):
    N, P, nst = 2048, 8, 120
    u0, dt = _sines(N, 0.05)
    a = gpu.Stepper(n=N, p=P, order=2, L=2, nu=0.05, dt=dt, nsteps_max=nst, seed=5)
    u, s = dev(u0), torch.empty(N, dtype=torch.float64, device="cuda")
    a.run(u, s, 50)
    snap = a.snapshot(u)
    a.run(u, s, nst - 50)
    ref = host(u)
    b = gpu.Stepper(n=N, p=P, order=2, L=2, nu=0.05, dt=dt, nsteps_max=nst, seed=5)
    v = torch.empty_like(u)
    b.restore(snap, v)                 # foreign buffer: the step is read from it
    assert b.n == 50
    b.run(v, s, nst - 50)
    assert np.array_equal(host(v), ref)
    a.restore(snap, v)                 # own buffer: the step comes from the host record
    assert a.n == 50
