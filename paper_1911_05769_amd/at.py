"""ctypes binding of libat.so (see include/at.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory (fields, workspace) and the stream.
The library must be built in-tree (``paper_1911_05769_amd/libat.so``); there is
no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import math
import os
import sys
from typing import Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libat.so")

AT_ABI_VERSION = 4
AT_MAX_SCALARS = 4
AT_OK, AT_ERR_ARG, AT_ERR_SHAPE, AT_ERR_DELAY, AT_ERR_HIP, AT_ERR_NOMEM, AT_ERR_STATE, \
    AT_ERR_TIMEOUT = 0, -1, -2, -3, -4, -5, -6, -7
DELAY_GENERATE, DELAY_HOST = 0, 1
DIST_UNIFORM, DIST_HALF_ZERO = 0, 1
DEBUG_POISON_RING = 1
STATUS_NAMES = {0: "AT_OK", -1: "AT_ERR_ARG", -2: "AT_ERR_SHAPE", -3: "AT_ERR_DELAY",
                -4: "AT_ERR_HIP", -5: "AT_ERR_NOMEM", -6: "AT_ERR_STATE",
                -7: "AT_ERR_TIMEOUT"}


class AtError(RuntimeError):
    def __init__(self, status: int, what: str, msg: str):
        super().__init__("%s: %s (%s)" % (what, STATUS_NAMES.get(status, status), msg))
        self.status = status


class Config(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("dim", ctypes.c_int32),
        ("n", ctypes.c_int64 * 3),
        ("p", ctypes.c_int32 * 3),
        ("order", ctypes.c_int32),
        ("L", ctypes.c_int32),
        ("halo_mode", ctypes.c_int32),
        ("adv_mode", ctypes.c_int32),
        ("nu", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("length", ctypes.c_double),
        ("adv_speed", ctypes.c_double),
        ("delay_mode", ctypes.c_int32),
        ("delay_dist", ctypes.c_int32),
        ("delay_seed", ctypes.c_uint64),
        ("delays_host", ctypes.c_void_p),
        ("nsteps_max", ctypes.c_int64),
        ("record", ctypes.c_int32),
        ("ckpt_every", ctypes.c_int32),
        ("fuse_steps", ctypes.c_int32),
        ("arith", ctypes.c_int32),
        ("nscalars", ctypes.c_int32),
        ("reserved1", ctypes.c_int32),
        ("alpha", ctypes.c_double * AT_MAX_SCALARS),
        ("stream", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p),
        ("workspace_bytes", ctypes.c_uint64),
    ]


_lib = None
_P = ctypes.c_void_p

# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "at_abi_version": (ctypes.c_int32, []),
    "at_last_error": (ctypes.c_char_p, []),
    "at_config_bytes": (ctypes.c_uint64, []),
    "at_workspace_bytes": (ctypes.c_int, [_P, _P]),
    "at_init": (ctypes.c_int, [_P, _P]),
    "at_free": (None, [_P]),
    "at_step": (ctypes.c_int, [_P, _P, _P]),
    "at_run": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64]),
    "at_run_ws": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64,
                                 ctypes.c_int64]),
    "at_ws_capacity": (ctypes.c_int, [_P, _P]),
    "at_autotune": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, _P]),
    "at_set_fuse": (ctypes.c_int, [_P, ctypes.c_int32]),
    "at_set_adjoint_fuse": (ctypes.c_int, [_P, ctypes.c_int32]),
    "at_set_variant": (ctypes.c_int, [_P, ctypes.c_int32]),
    "at_set_graph": (ctypes.c_int, [_P, ctypes.c_int32]),
    "at_set_debug": (ctypes.c_int, [_P, ctypes.c_int32]),
    "at_query": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "at_delays_copy": (ctypes.c_int, [_P, _P]),
    "at_snapshot_bytes": (ctypes.c_int, [_P, _P]),
    "at_snapshot": (ctypes.c_int, [_P, _P, _P]),
    "at_restore": (ctypes.c_int, [_P, _P, _P]),
    "at_stats": (ctypes.c_int, [_P, _P, _P]),
    "at_stats_noalloc": (ctypes.c_int, [_P, ctypes.c_int64, _P, _P]),
    "at_loss": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "at_adjoint": (ctypes.c_int, [_P, _P, _P, _P]),
    "at_batch_workspace_bytes": (ctypes.c_int, [_P, ctypes.c_int32, _P]),
    "at_batch_init": (ctypes.c_int, [_P, ctypes.c_int32, _P, ctypes.c_uint64, _P]),
    "at_batch_free": (None, [_P]),
    "at_batch_run": (ctypes.c_int, [_P, _P, _P, ctypes.c_int64, ctypes.c_int32]),
    "at_batch_autotune": (ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int32, _P]),
    "at_batch_set_fuse": (ctypes.c_int, [_P, ctypes.c_int32]),
    "at_batch_reset": (ctypes.c_int, [_P]),
    "at_batch_query": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "at_batch_set_variant": (ctypes.c_int, [_P, ctypes.c_int32]),
}


def lib():
    """Load libat.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libat.so not found at %s: build it with "
                               "`python -m paper_1911_05769_amd.build`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        if L.at_abi_version() != AT_ABI_VERSION:
            raise RuntimeError("libat.so ABI %d, binding expects %d" % (L.at_abi_version(),
                                                                       AT_ABI_VERSION))
        if L.at_config_bytes() != ctypes.sizeof(Config):
            raise RuntimeError("at_config layout mismatch: library %d bytes, binding %d" %
                               (L.at_config_bytes(), ctypes.sizeof(Config)))
        _lib = L
    return _lib


def _check(st: int, what: str):
    if st != AT_OK:
        raise AtError(st, what, lib().at_last_error().decode(errors="replace"))


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _require_f64_cuda(t: torch.Tensor, numel: int, what: str):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError("%s must be a CUDA float64 tensor" % what)
    if not t.is_contiguous() or t.numel() != numel:
        raise ValueError("%s must be contiguous with %d elements" % (what, numel))


def stats_noalloc(u: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
    """at_stats_noalloc on the current stream: (max|u|, mean u, sum|u|, count
    of non-finite values) of the CUDA float64 tensor u into the 4-element
    CUDA float64 tensor out, with no allocation by the library."""
    _require_f64_cuda(u, u.numel(), "u")
    _require_f64_cuda(out, 4, "out")
    stream = torch.cuda.current_stream(u.device).cuda_stream
    _check(lib().at_stats_noalloc(_ptr(u), u.numel(), _ptr(out), ctypes.c_void_p(stream)),
           "at_stats_noalloc")
    return out


def levels_for_order(order: int) -> int:
    return 2 if order == 2 else 3


def make_config(*, dim=1, n, p, order=2, L=0, nu, dt, nsteps_max, length=2 * math.pi,
                halo_mode=0, adv_mode=0, adv_speed=0.0, delays=None, seed=0,
                dist=DIST_UNIFORM, record=False, ckpt_every=0, fuse_steps=1,
                stream=None, arith=0, alpha=()) -> Config:
    """alpha: diffusivities of the passive scalars (3D only), one per scalar."""
    c = Config()
    c.abi_version = AT_ABI_VERSION
    c.dim = dim
    nn = list(n) + [1] * (3 - len(n)) if isinstance(n, (tuple, list)) else [n, 1, 1]
    pp = list(p) + [1] * (3 - len(p)) if isinstance(p, (tuple, list)) else [p, 1, 1]
    for a in range(3):
        c.n[a] = int(nn[a])
        c.p[a] = int(pp[a])
    c.order, c.L = int(order), int(L)
    c.halo_mode, c.adv_mode = int(halo_mode), int(adv_mode)
    c.nu, c.dt, c.length, c.adv_speed = float(nu), float(dt), float(length), float(adv_speed)
    c.delay_mode = DELAY_HOST if delays is not None else DELAY_GENERATE
    c.delay_dist = int(dist)
    c.delay_seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    c.delays_host = None
    c.nsteps_max = int(nsteps_max)
    c.record = 1 if record else 0
    c.ckpt_every = int(ckpt_every)
    c.fuse_steps = int(fuse_steps)
    c.arith = int(arith)
    al = [float(a) for a in alpha]
    if len(al) > AT_MAX_SCALARS:
        raise ValueError("at most %d passive scalars" % AT_MAX_SCALARS)
    c.nscalars = len(al)
    c.reserved1 = 0
    for j in range(AT_MAX_SCALARS):
        c.alpha[j] = al[j] if j < len(al) else 0.0
    c.stream = stream
    c.workspace = None
    c.workspace_bytes = 0
    return c


def workspace_bytes(cfg: Config) -> int:
    out = ctypes.c_uint64(0)
    _check(lib().at_workspace_bytes(ctypes.byref(cfg), ctypes.byref(out)), "at_workspace_bytes")
    return int(out.value)


def _alloc_workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns >= 512-byte aligned blocks
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise RuntimeError("workspace not 256-byte aligned")
    return ws


class Stepper:
    """One AT Burgers problem (1D scalar or 3D vector) on one device.

    Fields are torch float64 CUDA tensors: 1D shape (n,), 3D shape
    (3 + len(alpha), nz, ny, nx): the velocity, then the passive scalars with
    diffusivities ``alpha``.
    ``delays`` (int8 array [nsteps_max][F]) selects host mode; otherwise the
    library generates them from ``seed`` and ``dist``."""

    def __init__(self, *, dim=1, n, p, order=2, L=0, nu, dt, nsteps_max,
                 length=2 * math.pi, halo_mode=0, adv_mode=0, adv_speed=0.0, delays=None,
                 seed=0, dist=DIST_UNIFORM, record=False, ckpt_every=0, fuse_steps=1,
                 device="cuda", arith=0, alpha=()):
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.cfg = make_config(dim=dim, n=n, p=p, order=order, L=L, nu=nu, dt=dt,
                               nsteps_max=nsteps_max, length=length, halo_mode=halo_mode,
                               adv_mode=adv_mode, adv_speed=adv_speed, delays=delays,
                               seed=seed, dist=dist, record=record, ckpt_every=ckpt_every,
                               fuse_steps=fuse_steps, arith=arith, alpha=alpha,
                               stream=ctypes.c_void_p(self.stream.cuda_stream))
        self.dim = dim
        self.shape = (int(self.cfg.n[0]),) if dim == 1 else \
            (3 + int(self.cfg.nscalars), int(self.cfg.n[2]), int(self.cfg.n[1]),
             int(self.cfg.n[0]))
        self.numel = int(np.prod(self.shape))
        self.nfaces = (2 if dim == 1 else 6) * int(np.prod([self.cfg.p[a] for a in range(3)]))
        self._ctx = ctypes.c_void_p(None)
        self._delays_host = None
        if delays is not None:
            d = np.ascontiguousarray(delays, dtype=np.int8)
            if d.shape != (nsteps_max, self.nfaces):
                raise ValueError("delays must have shape (%d, %d)" % (nsteps_max, self.nfaces))
            self._delays_host = d
            self.cfg.delays_host = d.ctypes.data_as(ctypes.c_void_p)
        self.workspace = _alloc_workspace(workspace_bytes(self.cfg), self.device)
        self.cfg.workspace = ctypes.c_void_p(self.workspace.data_ptr())
        self.cfg.workspace_bytes = self.workspace.numel()
        _check(lib().at_init(ctypes.byref(self.cfg), ctypes.byref(self._ctx)), "at_init")
        self.cfg.delays_host = None

    def close(self):
        """Release the library handle (host memory only; the workspace tensor
        is freed with this object).  Idempotent."""
        if getattr(self, "_ctx", None):
            lib().at_free(self._ctx)
            self._ctx = ctypes.c_void_p(None)

    def __del__(self, _finalizing=sys.is_finalizing):
        # never call into the library while the interpreter shuts down: the
        # HIP runtime may already be tearing itself down by then (the check is
        # bound at definition time: module globals may be gone at exit)
        try:
            if not _finalizing():
                self.close()
        except Exception:
            pass

    # -- fields ------------------------------------------------------------
    def empty(self) -> torch.Tensor:
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    def _f(self, t, what):
        _require_f64_cuda(t, self.numel, what)
        return _ptr(t)

    # -- stepping ----------------------------------------------------------
    def step(self, u_in: torch.Tensor, u_out: torch.Tensor):
        _check(lib().at_step(self._ctx, self._f(u_in, "u_in"), self._f(u_out, "u_out")),
               "at_step")

    def run(self, u: torch.Tensor, scratch: torch.Tensor, nsteps: int):
        _check(lib().at_run(self._ctx, self._f(u, "u"), self._f(scratch, "scratch"),
                            int(nsteps)), "at_run")

    def run_ws(self, u: torch.Tensor, nsteps: int, jitter: int = 0, seed: int = 0,
               spin_limit: int = 0, scratch: torch.Tensor = None):
        """Weakly-synchronous run with emergent delays (see at_run_ws); the
        delays used are returned afterwards by delays().  3D needs a scratch
        field (allocated here when not given)."""
        if self.dim == 3 and scratch is None:
            scratch = self.empty()
        scr = self._f(scratch, "scratch") if scratch is not None else None
        _check(lib().at_run_ws(self._ctx, self._f(u, "u"), scr, int(nsteps), int(jitter),
                               int(seed) & 0xFFFFFFFFFFFFFFFF, int(spin_limit)), "at_run_ws")

    def ws_capacity(self) -> int:
        """Largest tile count a weakly-synchronous run of this shape can use."""
        out = ctypes.c_int64(0)
        _check(lib().at_ws_capacity(self._ctx, ctypes.byref(out)), "at_ws_capacity")
        return int(out.value)

    def autotune(self, u0: torch.Tensor, trial_steps: int) -> int:
        t1, t2 = self.empty(), self.empty()
        out = ctypes.c_int32(0)
        _check(lib().at_autotune(self._ctx, self._f(u0, "u0"), _ptr(t1), _ptr(t2),
                                 int(trial_steps), ctypes.byref(out)), "at_autotune")
        return int(out.value)

    def set_fuse(self, s: int):
        _check(lib().at_set_fuse(self._ctx, int(s)), "at_set_fuse")

    def set_adjoint_fuse(self, s: int):
        """Reverse steps per adjoint launch: 0 automatic, 1 one step per launch."""
        _check(lib().at_set_adjoint_fuse(self._ctx, int(s)), "at_set_adjoint_fuse")

    def set_variant(self, v: int):
        """Kernel variant (see at_set_variant).  1D: 0 automatic, 1/2/3 = 16/8/4
        points per thread in fused launches, 4 = the whole grid in one
        workgroup (one launch per run; small grids only)."""
        _check(lib().at_set_variant(self._ctx, int(v)), "at_set_variant")

    def set_graph(self, on: bool = True):
        """Replay run() from a captured HIP graph (see at_set_graph)."""
        _check(lib().at_set_graph(self._ctx, 1 if on else 0), "at_set_graph")

    def set_debug(self, flags: int):
        """AT_DEBUG_* flags, e.g. DEBUG_POISON_RING (see at_set_debug)."""
        _check(lib().at_set_debug(self._ctx, int(flags)), "at_set_debug")

    def query(self):
        """(step n, steps per launch, ring levels R)"""
        n, s, R = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().at_query(self._ctx, ctypes.byref(n), ctypes.byref(s), ctypes.byref(R),
                              None), "at_query")
        return int(n.value), int(s.value), int(R.value)

    @property
    def variant(self) -> int:
        """Kernel variant in use (1D: 0 automatic, 1/2/3 = 16/8/4 points per thread,
        4 = the whole grid in one workgroup)."""
        v = ctypes.c_int32()
        _check(lib().at_query(self._ctx, None, None, None, ctypes.byref(v)), "at_query")
        return int(v.value)

    @property
    def n(self) -> int:
        return self.query()[0]

    def delays(self) -> np.ndarray:
        out = np.empty((int(self.cfg.nsteps_max), self.nfaces), dtype=np.int8)
        _check(lib().at_delays_copy(self._ctx, out.ctypes.data_as(ctypes.c_void_p)),
               "at_delays_copy")
        return out

    # -- state -------------------------------------------------------------
    def snapshot(self, u: torch.Tensor) -> torch.Tensor:
        nb = ctypes.c_uint64(0)
        _check(lib().at_snapshot_bytes(self._ctx, ctypes.byref(nb)), "at_snapshot_bytes")
        buf = _alloc_workspace(int(nb.value), self.device)
        _check(lib().at_snapshot(self._ctx, self._f(u, "u"), _ptr(buf)), "at_snapshot")
        return buf

    def restore(self, buf: torch.Tensor, u: torch.Tensor):
        _check(lib().at_restore(self._ctx, _ptr(buf), self._f(u, "u")), "at_restore")

    # -- reductions, loss, adjoint -----------------------------------------
    def stats(self, u: torch.Tensor) -> torch.Tensor:
        """(max|u|, mean u, sum|u|, count of non-finite values) on the device;
        max|u| is NaN when any value is NaN."""
        out = torch.empty(4, dtype=torch.float64, device=self.device)
        _check(lib().at_stats(self._ctx, self._f(u, "u"), _ptr(out)), "at_stats")
        return out

    def loss(self, u: torch.Tensor, target: torch.Tensor, lam: Optional[torch.Tensor] = None):
        J = torch.empty(1, dtype=torch.float64, device=self.device)
        if lam is not None:
            self._f(lam, "lam")
        _check(lib().at_loss(self._ctx, self._f(u, "u"), self._f(target, "target"), _ptr(lam),
                             _ptr(J)), "at_loss")
        return J

    def adjoint(self, lam_T: torch.Tensor):
        g = self.empty()
        gnu = torch.empty(1, dtype=torch.float64, device=self.device)
        _check(lib().at_adjoint(self._ctx, self._f(lam_T, "lambda_T"), _ptr(g), _ptr(gnu)),
               "at_adjoint")
        return g, gnu


class Batch:
    """Many independent 1D instances advanced by the same launches."""

    def __init__(self, instances: Sequence[dict], device="cuda", fuse_steps=1):
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        cfgs = (Config * len(instances))()
        self._keep = []
        for j, ins in enumerate(instances):
            kw = dict(ins)
            delays = kw.pop("delays", None)
            c = make_config(dim=1, fuse_steps=fuse_steps,
                            stream=ctypes.c_void_p(self.stream.cuda_stream), delays=delays, **kw)
            if delays is not None:
                d = np.ascontiguousarray(delays, dtype=np.int8)
                self._keep.append(d)
                c.delays_host = d.ctypes.data_as(ctypes.c_void_p)
            cfgs[j] = c
        self.count = len(instances)
        self.sizes = [int(cfgs[j].n[0]) for j in range(self.count)]
        nb = ctypes.c_uint64(0)
        _check(lib().at_batch_workspace_bytes(cfgs, self.count, ctypes.byref(nb)),
               "at_batch_workspace_bytes")
        self.workspace = _alloc_workspace(int(nb.value), self.device)
        self._h = ctypes.c_void_p(None)
        _check(lib().at_batch_init(cfgs, self.count, _ptr(self.workspace),
                                   self.workspace.numel(), ctypes.byref(self._h)),
               "at_batch_init")
        self._keep = []

    @classmethod
    def from_workloads(cls, wls, device="cuda", fuse_steps=1, arith=0):
        """Instances from inputs.Workload objects (1D)."""
        ins = [dict(n=w.n[0], p=w.p[0], order=w.order, L=w.L, nu=w.nu, dt=w.dt,
                    nsteps_max=w.nsteps, seed=w.seed, dist=w.dist, length=w.length, arith=arith)
               for w in wls]
        return cls(ins, device=device, fuse_steps=fuse_steps)

    def close(self):
        """Release the batch handle, its cached graph and capture stream.
        Idempotent."""
        if getattr(self, "_h", None):
            lib().at_batch_free(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self, _finalizing=sys.is_finalizing):
        try:
            if not _finalizing():
                self.close()
        except Exception:
            pass

    def _ptrs(self, fields, what):
        if len(fields) != self.count:
            raise ValueError("%s: need %d fields" % (what, self.count))
        arr = (ctypes.c_void_p * self.count)()
        for j, t in enumerate(fields):
            _require_f64_cuda(t, self.sizes[j], "%s[%d]" % (what, j))
            arr[j] = t.data_ptr()
        return arr

    def run(self, u, scratch, nsteps: int, use_graph: bool = False):
        _check(lib().at_batch_run(self._h, self._ptrs(u, "u"), self._ptrs(scratch, "scratch"),
                                  int(nsteps), 1 if use_graph else 0), "at_batch_run")

    def autotune(self, u0, trial_steps: int) -> int:
        t1 = [torch.empty_like(x) for x in u0]
        t2 = [torch.empty_like(x) for x in u0]
        out = ctypes.c_int32(0)
        _check(lib().at_batch_autotune(self._h, self._ptrs(u0, "u0"), self._ptrs(t1, "t1"),
                                       self._ptrs(t2, "t2"), int(trial_steps),
                                       ctypes.byref(out)), "at_batch_autotune")
        return int(out.value)

    def set_fuse(self, s: int):
        _check(lib().at_batch_set_fuse(self._h, int(s)), "at_batch_set_fuse")

    def reset(self):
        _check(lib().at_batch_reset(self._h), "at_batch_reset")

    def query(self):
        """(shared step n, steps per launch, its limit)"""
        n, s, m = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().at_batch_query(self._h, ctypes.byref(n), ctypes.byref(s), ctypes.byref(m),
                                    None), "at_batch_query")
        return int(n.value), int(s.value), int(m.value)

    @property
    def variant(self) -> int:
        """Points-per-thread variant (0/1: 16, 2: 8, 3: 4)."""
        v = ctypes.c_int32()
        _check(lib().at_batch_query(self._h, None, None, None, ctypes.byref(v)),
               "at_batch_query")
        return int(v.value)

    def set_variant(self, v: int):
        _check(lib().at_batch_set_variant(self._h, int(v)), "at_batch_set_variant")
