"""CPU oracle for the asynchrony-tolerant (AT) Burgers stepper.

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline
leg of the benchmark are the only callers.  Nothing in the GPU library imports,
links or executes anything here, and this package imports nothing from it.

``liboracle.so`` (built from ``at_oracle.c`` by ``oracle/build.py``) holds the
plain C implementation; ``oracle.twin`` is a vectorised NumPy restatement with
full-grid history that also runs in complex arithmetic (complex-step
derivatives).  Both follow the paper's section 2 (delays, AT schemes,
Eqs. (1)-(2)), section 3 (Burgers equations, Eq. (4); central differences and
forward Euler) and section 5.2 (AT = halo approximation + unchanged stencil).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_int = ctypes.c_int
_dbl = ctypes.c_double
_u64 = ctypes.c_uint64
_p = ctypes.c_void_p


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_delays.argtypes = [_i64, _i64, _int, _int, _int, _u64, _p]
        L.or_check_delays.argtypes = [_i64, _i64, _int, _int, _p]
        L.or_splitmix_sequence.argtypes = [_u64, _i64, _p]
        L.or_splitmix_sequence.restype = _u64
        L.or_halo.argtypes = [_int, _int, _int, _p]
        L.or_halo.restype = _dbl
        L.or_run1d.argtypes = [_i64, _i64, _int, _int, _int, _int, _dbl, _dbl, _dbl, _dbl,
                               _p, _i64, _p, _p]
        L.or_adjoint1d.argtypes = [_i64, _i64, _int, _int, _int, _int, _dbl, _dbl, _dbl, _dbl,
                                   _p, _i64, _p, _p, _p, _p]
        L.or_run3d.argtypes = [_p, _p, _int, _int, _dbl, _dbl, _dbl, _p, _i64, _p, _p]
        L.or_run3ds.argtypes = [_p, _p, _int, _p, _int, _int, _dbl, _dbl, _dbl, _p, _i64, _p,
                                _p]
        L.or_set_threads.argtypes = [_int]
        L.or_set_threads.restype = None
        L.or_max_threads.argtypes = []
        L.or_max_threads.restype = _int
        L.or_stats.argtypes = [_i64, _p, _p]
        L.or_stats.restype = None
        L.or_loss.argtypes = [_i64, _p, _p, _p]
        L.or_loss.restype = _dbl
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(st, what):
    if st != 0:
        raise OracleError("%s failed with status %d" % (what, st))


def levels_for_order(order: int) -> int:
    """m, the number of time levels an AT halo value is extrapolated from."""
    return 2 if order == 2 else 3


def splitmix_sequence(seed: int, count: int) -> np.ndarray:
    out = np.empty(count, dtype=np.uint64)
    lib().or_splitmix_sequence(_u64(seed), count, _ptr(out))
    return out


def delays(nsteps: int, nfaces: int, L: int, m: int, dist: int, seed: int) -> np.ndarray:
    """int8 delays k[n][f] (after the start-up clamp)."""
    k = np.empty((nsteps, nfaces), dtype=np.int8)
    _check(lib().or_delays(nsteps, nfaces, L, m, dist, _u64(seed), _ptr(k)), "or_delays")
    return k


def check_delays(k: np.ndarray, L: int, m: int) -> bool:
    k = np.ascontiguousarray(k, dtype=np.int8)
    return lib().or_check_delays(k.shape[0], k.shape[1], L, m, _ptr(k)) == 0


def halo(kk: int, m: int, values, stale: bool = False) -> float:
    v = np.zeros(3, dtype=np.float64)
    v[:len(values)] = values
    return lib().or_halo(kk, m, 1 if stale else 0, _ptr(v))


def run1d(u0, N, P, order, L, nu, dt, k, nsteps, length=2 * np.pi, stale=False,
          linear=False, adv_speed=0.0) -> np.ndarray:
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    k = np.ascontiguousarray(k, dtype=np.int8)
    assert u0.shape == (N,) and k.shape[0] >= nsteps and k.shape[1] == 2 * P
    out = np.empty(N, dtype=np.float64)
    st = lib().or_run1d(N, P, order, L, 1 if stale else 0, 1 if linear else 0, nu, dt,
                        length, adv_speed, _ptr(k), nsteps, _ptr(u0), _ptr(out))
    _check(st, "or_run1d")
    return out


def adjoint1d(u0, lamT, N, P, order, L, nu, dt, k, nsteps, length=2 * np.pi, stale=False,
              linear=False, adv_speed=0.0):
    """(dJ/du0, dJ/dnu) for dJ/du(T) = lamT, dt fixed."""
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    lamT = np.ascontiguousarray(lamT, dtype=np.float64)
    k = np.ascontiguousarray(k, dtype=np.int8)
    lam0 = np.empty(N, dtype=np.float64)
    gnu = np.zeros(1, dtype=np.float64)
    st = lib().or_adjoint1d(N, P, order, L, 1 if stale else 0, 1 if linear else 0, nu, dt,
                            length, adv_speed, _ptr(k), nsteps, _ptr(u0), _ptr(lamT),
                            _ptr(lam0), _ptr(gnu))
    _check(st, "or_adjoint1d")
    return lam0, float(gnu[0])


def run3d(u0, n, p, L, nu, dt, k, nsteps, length=2 * np.pi, stale=False,
          alpha=()) -> np.ndarray:
    """u0: [3 + len(alpha)][nz][ny][nx]; n, p: (x, y, z) sizes and block counts.

    Components 0..2 are the velocity (diffusivity nu); each further component
    is a passive scalar advected by it with diffusivity alpha[s] (section 3.1,
    Eq. (4)).
    """
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    k = np.ascontiguousarray(k, dtype=np.int8)
    nx = np.asarray(n, dtype=np.int64)
    px = np.asarray(p, dtype=np.int64)
    al = np.ascontiguousarray(alpha, dtype=np.float64).reshape(-1)
    assert u0.shape == (3 + al.size, n[2], n[1], n[0])
    out = np.empty_like(u0)
    if al.size == 0:
        st = lib().or_run3d(_ptr(nx), _ptr(px), L, 1 if stale else 0, nu, dt, length, _ptr(k),
                            nsteps, _ptr(u0), _ptr(out))
        _check(st, "or_run3d")
    else:
        st = lib().or_run3ds(_ptr(nx), _ptr(px), al.size, _ptr(al), L, 1 if stale else 0, nu,
                             dt, length, _ptr(k), nsteps, _ptr(u0), _ptr(out))
        _check(st, "or_run3ds")
    return out


def set_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (results do not depend on it)."""
    lib().or_set_threads(int(n))


def max_threads() -> int:
    return int(lib().or_max_threads())


def stats(u) -> tuple:
    """(max|u|, mean u, sum|u|, count of non-finite values) with serial
    Neumaier sums; max|u| is NaN when any value is NaN."""
    u = np.ascontiguousarray(u, dtype=np.float64).ravel()
    out = np.empty(4, dtype=np.float64)
    lib().or_stats(u.size, _ptr(u), _ptr(out))
    return float(out[0]), float(out[1]), float(out[2]), int(out[3])


def loss(u, target):
    """(J, lam) with J = 0.5 sum (u - target)^2, lam = u - target."""
    u = np.ascontiguousarray(u, dtype=np.float64).ravel()
    t = np.ascontiguousarray(target, dtype=np.float64).ravel()
    lam = np.empty_like(u)
    J = lib().or_loss(u.size, _ptr(u), _ptr(t), _ptr(lam))
    return J, lam
