"""at_stats_noalloc, the allocation-free variant of at_stats for callers that
cannot allocate device memory (its per-workgroup partials live in a static
device array): called through the C ABI, it gives the same four outputs as
at_stats on the same input, bit for bit (the same kernels in the same order),
on two calls in a row, the second with a smaller input; sizes outside
1..AT_NOALLOC_MAX_POINTS are refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _noalloc(gpu, u, n, out):
    stream = torch.cuda.current_stream().cuda_stream
    return gpu.lib().at_stats_noalloc(ctypes.c_void_p(u.data_ptr()), n,
                                      ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stream))


def test_stats_noalloc_equals_at_stats(gpu):
    g = np.random.default_rng(17)
    for i, n in enumerate(((1 << 22) + 3, 1000)):       # the second call is smaller
        x = g.standard_normal(n) * 10.0 ** g.uniform(-3, 3, n)
        if i == 1:
            x[17] = np.nan
            x[999] = np.inf
        u = _dev(x)
        st = gpu.Stepper(n=n, p=1, order=2, L=0, nu=0.0, dt=1.0, nsteps_max=1)
        ref = st.stats(u).cpu().numpy()
        out = torch.full((4,), -7.0, dtype=torch.float64, device="cuda")
        assert _noalloc(gpu, u, n, out) == gpu.AT_OK
        got = out.cpu().numpy()
        print("call %d, n = %d: noalloc %r, at_stats %r" % (i, n, got.tolist(), ref.tolist()),
              flush=True)
        assert np.array_equal(got, ref, equal_nan=True)
        assert got[3] == (2 if i == 1 else 0)
        st.close()


def test_stats_noalloc_refuses_bad_sizes(gpu):
    u = torch.zeros(8, dtype=torch.float64, device="cuda")
    out = torch.full((4,), -7.0, dtype=torch.float64, device="cuda")
    for n in (0, -1, (1 << 40) + 1):
        assert _noalloc(gpu, u, n, out) == gpu.AT_ERR_ARG
        assert "at_stats_noalloc" in gpu.lib().at_last_error().decode()
    torch.cuda.synchronize()
    assert bool((out == -7.0).all())
