"""torch.autograd binding of the unrolled-ADMM derivative (argument marshalling only).

    plan = Plan(coil, mask, mu=0.1, prior="tv")
    unrolled = Unrolled(plan, iters=20, ckpt_every=5)
    x = unrolled(y, lam, mu)          # y complex64 k-space; lam, mu 0-dim float tensors or floats
    loss(x).backward()                # fills y.grad, lam.grad, mu.grad

Forward and backward both run in libcsmri (cs_admm_forward_ckpt /
cs_admm_backward): K iterations of Algorithm 2 (plan prior "tv") or
Algorithm 1 (prior "dft") with checkpoints every
`ckpt_every` iterations, then the reverse sweep.  Complex gradients follow
torch's convention (dL/dRe + i dL/dIm).  One Unrolled object holds the
checkpoints of its latest forward: a backward must follow its own forward
before the object runs another (checked; use one object per pending graph).
"""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import check
from .api import Plan, _need, _ptr, _stream


class Unrolled:
    """Differentiable K-iteration reconstruction (temporal TV or temporal DFT) on a plan."""

    def __init__(self, plan: Plan, iters: int, ckpt_every: int = 5):
        if plan.prior not in ("tv", "dft"):
            raise ValueError("the unrolled derivative is implemented for the temporal TV and DFT priors")
        self.plan = plan
        self.iters = int(iters)
        self.ckpt_every = int(ckpt_every)
        h = ctypes.c_void_p()
        check(_lib.load().cs_grad_create(plan.handle, self.iters, self.ckpt_every, ctypes.byref(h)),
              "cs_grad_create")
        self._h = h
        self.generation = 0
        self._pending = None

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            _lib.load().cs_grad_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h or not self._h.value:
            raise RuntimeError("Unrolled is closed")
        return self._h

    # -- raw calls (no autograd)
    def forward_raw(self, y: torch.Tensor, lam: float, mu: float, stream=None) -> torch.Tensor:
        _need(y, "y", torch.complex64, self.plan.kspace_shape)
        x = torch.empty(self.plan.image_shape, dtype=torch.complex64, device=y.device)
        check(_lib.load().cs_admm_forward_ckpt(self.handle, _ptr(y), float(lam), float(mu), _ptr(x),
                                               _stream(stream)), "cs_admm_forward_ckpt")
        self.plan.mu = float(mu)
        self.generation += 1
        return x

    def backward_raw(self, grad_x: torch.Tensor, stream=None):
        """Returns (dL/dy, tensor([dL/dlambda, dL/dmu])) for dL/dx_K = grad_x."""
        grad_x = grad_x.contiguous()
        _need(grad_x, "grad_x", torch.complex64, self.plan.image_shape)
        gy = torch.empty(self.plan.kspace_shape, dtype=torch.complex64, device=grad_x.device)
        gs = torch.empty(2, dtype=torch.float32, device=grad_x.device)
        check(_lib.load().cs_admm_backward(self.handle, _ptr(grad_x), _ptr(gy), _ptr(gs), _stream(stream)),
              "cs_admm_backward")
        return gy, gs

    def __call__(self, y: torch.Tensor, lam, mu) -> torch.Tensor:
        lam_t = lam if isinstance(lam, torch.Tensor) else torch.tensor(float(lam))
        mu_t = mu if isinstance(mu, torch.Tensor) else torch.tensor(float(mu))
        return _UnrolledFn.apply(y, lam_t, mu_t, self)


class _UnrolledFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, lam, mu, unrolled: Unrolled):
        x = unrolled.forward_raw(y.detach(), float(lam), float(mu))
        ctx.unrolled = unrolled
        ctx.generation = unrolled.generation
        ctx.lam_meta = (lam.shape, lam.dtype, lam.device)
        ctx.mu_meta = (mu.shape, mu.dtype, mu.device)
        return x

    @staticmethod
    def backward(ctx, grad_x):
        u = ctx.unrolled
        if u.generation != ctx.generation:
            raise RuntimeError("this Unrolled object ran another forward before this backward; "
                               "use one Unrolled object per pending backward")
        gy, gs = u.backward_raw(grad_x)
        lshape, ldtype, ldev = ctx.lam_meta
        mshape, mdtype, mdev = ctx.mu_meta
        glam = gs[0].to(device=ldev, dtype=ldtype).reshape(lshape) if ctx.needs_input_grad[1] else None
        gmu = gs[1].to(device=mdev, dtype=mdtype).reshape(mshape) if ctx.needs_input_grad[2] else None
        return (gy if ctx.needs_input_grad[0] else None), glam, gmu, None
