"""Differentiable KDK trajectory: forward through nbody_step with checkpoints,
backward through the library's hand-written adjoint sweep (nbody_traj_grad).

Only (x, v) every `every` steps are kept on the device; the backward pass
recomputes each segment from its checkpoint with the same kernels as the
forward (bitwise the same trajectory) and sweeps it in reverse.

The sweep may run in another precision than the forward pass
(`adjoint_precision`): with an FP64 forward and an FP32C sweep the gradient is
that of the FP64 trajectory (each segment restarts from an FP64 checkpoint, so
the FP32C recompute stays within its 20-odd steps of it), at the cost of the
FP32C adjoint.
"""
from __future__ import annotations

import torch

from . import _binding as B


class NBodyTrajectory(torch.autograd.Function):
    """(x0, v0, m) -> (x_T, v_T) after `nsteps` KDK steps of size dt.

    Usage: xT, vT = NBodyTrajectory.apply(x0, v0, m, dt, nsteps, every, G, eps, precision[, adjoint_precision])
    x0, v0: (3, N) float64 CUDA tensors; m: (N,).  Gradients flow to all three.
    adjoint_precision (default: precision) is the pair arithmetic of the reverse sweep.
    """

    @staticmethod
    def forward(ctx, x0, v0, m, dt, nsteps, every=20, G=1.0, eps=0.01, precision="fp32c", adjoint_precision=None):
        nsteps, every = int(nsteps), int(every)
        if every < 1:
            raise ValueError("every must be >= 1")
        n = m.shape[0]
        nck = max(1, -(-nsteps // every))
        ckx = torch.empty((nck, 3, n), dtype=torch.float64, device=x0.device)
        ckv = torch.empty_like(ckx)
        x = x0.detach().contiguous().clone()
        v = v0.detach().contiguous().clone()
        md = m.detach().contiguous()
        a = torch.empty_like(x)
        done = 0
        for seg in range(nck):
            ckx[seg].copy_(x)
            ckv[seg].copy_(v)
            steps = min(every, nsteps - done)
            B.nbody_step(x, v, a, md, dt, steps, G=G, eps=eps, precision=precision, acc_valid=seg > 0)
            done += steps
        ctx.save_for_backward(ckx, ckv, md)
        ctx.cfg = (float(dt), nsteps, every, float(G), float(eps), adjoint_precision or precision)
        return x, v

    @staticmethod
    def backward(ctx, gxT, gvT):
        ckx, ckv, m = ctx.saved_tensors
        dt, nsteps, every, G, eps, precision = ctx.cfg
        if gxT is None:
            gxT = torch.zeros_like(ckx[0])
        if gvT is None:
            gvT = torch.zeros_like(ckx[0])
        gx0, gv0, gm = B.nbody_traj_grad(ckx, ckv, every, nsteps, m, dt, gxT.contiguous(), gvT.contiguous(),
                                         G=G, eps=eps, precision=precision)
        return gx0, gv0, gm, None, None, None, None, None, None, None


def trajectory(x0, v0, m, dt, nsteps, every=20, G=1.0, eps=0.01, precision="fp32c", adjoint_precision=None):
    """Functional form of NBodyTrajectory.apply."""
    return NBodyTrajectory.apply(x0, v0, m, dt, nsteps, every, G, eps, precision, adjoint_precision)
