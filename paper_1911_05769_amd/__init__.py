"""MI355X (gfx950) implementation of the asynchrony-tolerant (AT) explicit
Burgers stepper of arXiv:1911.05769 (weakly-synchronous PDE solver).

Submodules:
  at        ctypes binding of libat.so (C ABI in include/at.h)
  autograd  torch.autograd.Function over the stepper and its discrete adjoint
  inputs    seeded synthetic initial fields and workload parameters
  build     in-tree build of libat.so with hipcc (gfx950)
"""
__all__ = ["at", "autograd", "inputs", "build"]
