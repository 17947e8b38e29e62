"""Host-only checks of the C ABI: the library loads, exports every function
include/at.h declares, agrees on the at_config layout, and rejects invalid
configurations and delay arrays before touching a device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1911_05769_amd import at

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "at.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(at_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 20
    L = at.lib()
    for name in names:
        assert hasattr(L, name), name
    assert set(names) <= set(at.SIGNATURES) | {"at_config_bytes"}


def test_config_layout_and_version():
    L = at.lib()
    assert L.at_abi_version() == at.AT_ABI_VERSION
    assert L.at_config_bytes() == ctypes.sizeof(at.Config)


def _ws(**kw):
    base = dict(n=1024, p=8, order=2, L=2, nu=0.05, dt=1e-4, nsteps_max=10)
    base.update(kw)
    return at.workspace_bytes(at.make_config(**base))


@pytest.mark.parametrize("kw,status", [
    (dict(order=3), at.AT_ERR_ARG),
    (dict(p=7), at.AT_ERR_SHAPE),
    (dict(n=16, p=16), at.AT_ERR_SHAPE),             # tile narrower than 2h
    (dict(order=4, n=24, p=8), at.AT_ERR_SHAPE),     # W = 3 < 4
    (dict(L=16), at.AT_ERR_ARG),
    (dict(nu=-1.0), at.AT_ERR_ARG),
    (dict(dt=0.0), at.AT_ERR_ARG),
    (dict(dt=float("nan")), at.AT_ERR_ARG),
    (dict(fuse_steps=65), at.AT_ERR_ARG),
    (dict(record=True, ckpt_every=0), at.AT_ERR_ARG),
    (dict(dim=3, n=(16, 16, 16), p=(2, 2, 2), order=4), at.AT_ERR_ARG),
    (dict(adv_mode=2), at.AT_ERR_ARG),
    (dict(arith=2), at.AT_ERR_ARG),
    (dict(dim=3, n=(16, 16, 16), p=(2, 2, 2), order=2, arith=1), at.AT_ERR_ARG),
    (dict(alpha=(0.01,)), at.AT_ERR_ARG),                       # scalars are 3D only
    (dict(dim=3, n=(16, 16, 16), p=(2, 2, 2), alpha=(0.01, -1.0)), at.AT_ERR_ARG),
    (dict(dim=3, n=(16, 16, 16), p=(2, 2, 2), alpha=(float("inf"),)), at.AT_ERR_ARG),
])
def test_invalid_configs_rejected(kw, status):
    with pytest.raises(at.AtError) as e:
        _ws(**kw)
    assert e.value.status == status


def test_scalar_count_bounds_and_reserved_field():
    cfg = at.make_config(dim=3, n=(16, 16, 16), p=(2, 2, 2), nu=0.05, dt=1e-4, nsteps_max=4)
    out = ctypes.c_uint64(0)
    cfg.nscalars = at.AT_MAX_SCALARS + 1
    assert at.lib().at_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == at.AT_ERR_ARG
    cfg.nscalars = 1
    cfg.reserved1 = 7
    assert at.lib().at_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)) == at.AT_ERR_ARG
    with pytest.raises(ValueError):
        at.make_config(dim=3, n=(16, 16, 16), p=(2, 2, 2), nu=0.05, dt=1e-4, nsteps_max=4,
                       alpha=(0.1,) * (at.AT_MAX_SCALARS + 1))


def test_scalar_ring_grows_with_components():
    """The ring stores every component of each block face: (3 + s) / 3 times
    the velocity-only ring."""
    def ws(alpha):
        return _ws(dim=3, n=(32, 32, 32), p=(2, 2, 2), L=3, nsteps_max=1, alpha=alpha)
    w0, w2 = ws(()), ws((0.01, 0.02))
    assert w2 > w0


def test_workspace_sizes():
    plain = _ws()
    rec = _ws(record=True, ckpt_every=5)
    assert rec > plain > 0
    # 1D ring: R = L + m - 1 + 32 levels of 2P*h doubles
    big = _ws(n=1 << 24, p=4096, order=4, L=4, nsteps_max=2000)
    assert big >= 2000 * 8192 + (4 + 3 - 1 + 32) * 4096 * 2 * 2 * 8


def _init_with(delays, **kw):
    cfg = at.make_config(n=64, p=4, order=2, L=2, nu=0.05, dt=1e-4, nsteps_max=delays.shape[0],
                         delays=delays, **kw)
    d = np.ascontiguousarray(delays, np.int8)
    cfg.delays_host = d.ctypes.data_as(ctypes.c_void_p)
    cfg.workspace = ctypes.c_void_p(1 << 20)          # never dereferenced: rejected first
    cfg.workspace_bytes = at.workspace_bytes(cfg)
    ctx = ctypes.c_void_p()
    st = at.lib().at_init(ctypes.byref(cfg), ctypes.byref(ctx))
    return st, at.lib().at_last_error().decode()


def test_host_delays_validated_before_device_use():
    k = np.zeros((6, 8), np.int8)
    k[0, 3] = 1                      # level -1 would be read (m = 2 allows k <= n - 1)
    st, msg = _init_with(k)
    assert st == at.AT_ERR_DELAY and "k[0][3]" in msg
    k = np.zeros((6, 8), np.int8)
    k[5, 0] = 3                      # beyond L = 2
    st, _ = _init_with(k)
    assert st == at.AT_ERR_DELAY
    k[5, 0] = -1
    st, _ = _init_with(k)
    assert st == at.AT_ERR_DELAY


def test_workspace_checks():
    cfg = at.make_config(n=64, p=4, order=2, L=2, nu=0.05, dt=1e-4, nsteps_max=4)
    cfg.workspace = ctypes.c_void_p(1 << 20)
    cfg.workspace_bytes = 16
    ctx = ctypes.c_void_p()
    assert at.lib().at_init(ctypes.byref(cfg), ctypes.byref(ctx)) == at.AT_ERR_NOMEM
    cfg.workspace = ctypes.c_void_p((1 << 20) + 8)
    cfg.workspace_bytes = 1 << 30
    assert at.lib().at_init(ctypes.byref(cfg), ctypes.byref(ctx)) == at.AT_ERR_ARG
