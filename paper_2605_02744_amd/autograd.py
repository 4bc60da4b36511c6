"""Differentiable KDK trajectory: forward through nbody_step with checkpoints,
backward through the library's hand-written adjoint sweep (nbody_traj_grad).

Only (x, v) every `every` steps are kept on the device; the backward pass
recomputes each segment from its checkpoint with the same kernels as the
forward (bitwise the same trajectory) and sweeps it in reverse.

Two precisions are involved.  `precision` is the pair arithmetic of the
reverse sweep, where a gradient spends most of its time.  `forward_precision`
is that of the forward pass and its checkpoints, i.e. of the trajectory that
is differentiated.  By default an FP32C (or FP32) gradient differentiates the
FP64 trajectory: each segment of the sweep restarts from an FP64 checkpoint,
so its FP32C recompute stays within `every` steps of it, and the result is
the gradient of the FP64 map to FP32C accuracy.  An FP32C forward
(forward_precision="fp32c") differentiates the FP32C map instead, whose
sensitivities to single coordinates can differ from the FP64 map's by more
than the gradient tolerance of 1e-4 after a few hundred steps (mass
coordinates and small position components of the 16384-body, 200-step
workload: up to 4.7e-4); that form is cheaper (its forward runs in FP32C).
"""
from __future__ import annotations

import torch

from . import _binding as B


def _forward_default(precision, forward_precision):
    if forward_precision is not None:
        return forward_precision
    p = precision.lower() if isinstance(precision, str) else precision
    return "fp64" if p in ("fp32c", "fp32", B.NBODY_FP32C, B.NBODY_FP32) else precision


class NBodyTrajectory(torch.autograd.Function):
    """(x0, v0, m) -> (x_T, v_T) after `nsteps` KDK steps of size dt.

    Usage: xT, vT = NBodyTrajectory.apply(x0, v0, m, dt, nsteps, every, G, eps, precision[, forward_precision])
    x0, v0: (3, N) float64 CUDA tensors; m: (N,).  Gradients flow to all three.
    precision: pair arithmetic of the reverse sweep.  forward_precision: pair
    arithmetic of the forward pass (the differentiated trajectory); None means
    "fp64" for an FP32C/FP32 sweep and `precision` otherwise.
    """

    @staticmethod
    def forward(ctx, x0, v0, m, dt, nsteps, every=20, G=1.0, eps=0.01, precision="fp32c", forward_precision=None):
        nsteps, every = int(nsteps), int(every)
        if every < 1:
            raise ValueError("every must be >= 1")
        fprec = _forward_default(precision, forward_precision)
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
            B.nbody_step(x, v, a, md, dt, steps, G=G, eps=eps, precision=fprec, acc_valid=seg > 0)
            done += steps
        ctx.save_for_backward(ckx, ckv, md)
        ctx.cfg = (float(dt), nsteps, every, float(G), float(eps), precision)
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


def trajectory(x0, v0, m, dt, nsteps, every=20, G=1.0, eps=0.01, precision="fp32c", forward_precision=None):
    """Functional form of NBodyTrajectory.apply."""
    return NBodyTrajectory.apply(x0, v0, m, dt, nsteps, every, G, eps, precision, forward_precision)
