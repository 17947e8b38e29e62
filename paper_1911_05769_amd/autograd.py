"""torch.autograd.Function over the AT stepper and its hand-written discrete
adjoint (libat.so's at_run in record mode and at_adjoint).

    uT = AtBurgers.apply(u0, nu, spec)      # spec: StepSpec
    J = AtMisfit.apply(uT, target)          # 0.5 * ||uT - target||^2
    J.backward()                            # u0.grad, nu.grad via the adjoint

Gradients are those of the discrete map with dt held fixed: the same delay
array is replayed, and the forward keeps a checkpoint every ``ckpt_every``
steps from which the reverse sweep recomputes each segment.  The forward
advances ``fuse_steps`` steps per launch (the library lowers it to what the
grid allows); the adjoint's reverse launches are fused as far as the grid
allows.  All work runs on the stream that is current when the function is
applied.
"""
from __future__ import annotations

import dataclasses
import math

import torch

from . import at


@dataclasses.dataclass(frozen=True)
class StepSpec:
    n: int
    p: int
    order: int
    L: int
    dt: float
    nsteps: int
    ckpt_every: int
    seed: int = 0
    dist: int = at.DIST_UNIFORM
    length: float = 2 * math.pi
    halo_mode: int = 0
    fuse_steps: int = 64       # steps per forward launch (clamped to the grid's limit)


class AtBurgers(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0: torch.Tensor, nu: torch.Tensor, spec: StepSpec):
        st = at.Stepper(n=spec.n, p=spec.p, order=spec.order, L=spec.L, nu=float(nu),
                        dt=spec.dt, nsteps_max=spec.nsteps, length=spec.length,
                        halo_mode=spec.halo_mode, seed=spec.seed, dist=spec.dist, record=True,
                        ckpt_every=spec.ckpt_every, fuse_steps=spec.fuse_steps,
                        device=u0.device)
        u = u0.detach().contiguous().clone()
        scratch = torch.empty_like(u)
        st.run(u, scratch, spec.nsteps)
        ctx.stepper = st
        ctx.nu_meta = (nu.shape, nu.device, nu.dtype)
        return u

    @staticmethod
    def backward(ctx, grad_uT: torch.Tensor):
        g, gnu = ctx.stepper.adjoint(grad_uT.contiguous())
        shape, device, dtype = ctx.nu_meta
        return g, gnu.reshape(shape).to(device=device, dtype=dtype), None


class AtMisfit(torch.autograd.Function):
    """J = 0.5 * sum (u - target)^2 by the library's compensated reduction."""

    @staticmethod
    def forward(ctx, u: torch.Tensor, target: torch.Tensor):
        n = u.numel()
        helper = _reducer(n, u.device)
        lam = torch.empty_like(u)
        J = helper.loss(u.contiguous(), target.contiguous(), lam)
        ctx.save_for_backward(lam)
        return J.reshape(())

    @staticmethod
    def backward(ctx, gJ: torch.Tensor):
        (lam,) = ctx.saved_tensors
        return lam * gJ, -lam * gJ


_reducers = {}


def _reducer(n: int, device) -> at.Stepper:
    """A minimal context whose only use is the reduction kernels, bound to the
    stream that is current now (a context launches on the stream it was made
    with, so one is kept per stream)."""
    device = torch.device(device)
    if device.index is None:
        device = torch.device(device.type, torch.cuda.current_device())
    key = (n, str(device), torch.cuda.current_stream(device).cuda_stream)
    if key not in _reducers:
        _reducers[key] = at.Stepper(n=n, p=1, order=2, L=0, nu=0.0, dt=1.0, nsteps_max=0,
                                    device=device)
    return _reducers[key]
