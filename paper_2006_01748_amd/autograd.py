"""Gradients through many explicit steps, as a ``torch.autograd.Function``.

``run(ctx, params, lam1, lam2, theta, u0, v0, w0, dt, nsteps)`` advances the state
nsteps forward-Euler steps of eq. (3) on the GPU and returns (u, v, w) at the end.
Gradients flow to the five parameters (delta1, rho2, Delta2, rho3, delta3), the
per-cell tensor description (lambda1, lambda2, theta) and the initial state; dt is
a constant.

Memory follows the square-root schedule: the forward pass stores the state every
``every`` steps (ceil(N/every) checkpoints, caller-owned torch memory), and the
backward pass recomputes one segment of ``every`` states at a time from its
checkpoint and runs the adjoint steps backwards through it (all inside the HIP
library, one call).  With every = ceil(sqrt(N)) this keeps about 2 sqrt(N) states
and costs one extra forward pass.
"""
from __future__ import annotations

import math

import torch


class FVRun(torch.autograd.Function):
    @staticmethod
    def forward(fctx, params, lam1, lam2, theta, u0, v0, w0, gg, dt, nsteps, every):
        gg.set_params(params.detach().cpu().tolist())
        gg.set_tensor_eig(lam1.detach().contiguous(), lam2.detach().contiguous(), theta.detach().contiguous())
        gg.set_state(u0.detach().contiguous(), v0.detach().contiguous(), w0.detach().contiguous())
        sb = gg.state_bytes()
        nck = -(-nsteps // every)
        ckpt = torch.empty(nck * sb, dtype=torch.uint8, device=u0.device)
        gg.step_checkpointed(dt, nsteps, every, ckpt)
        outs = [torch.empty((gg.ny, gg.nx), dtype=u0.dtype, device=u0.device) for _ in range(3)]
        gg.get_state(out=outs)
        fctx.save_for_backward(params, lam1, lam2, theta)
        fctx.ckpt = ckpt
        fctx.gg = gg
        fctx.dt = dt
        fctx.nsteps = nsteps
        fctx.every = every
        return tuple(outs)

    @staticmethod
    def backward(fctx, gu, gv, gw):
        params, lam1, lam2, theta = fctx.saved_tensors
        if fctx.ckpt is None:
            raise RuntimeError("a second backward through the same run is not supported: the first released "
                               "its checkpoints (run the forward again)")
        gg = fctx.gg
        # the context may have been used in between: restore what this run used
        gg.set_params(params.detach().cpu().tolist())
        l1, l2, th = (x.detach().contiguous() for x in (lam1, lam2, theta))
        gg.set_tensor_eig(l1, l2, th)
        ref = l1
        lam = [(g if g is not None else torch.zeros_like(ref)).detach().to(ref.dtype).contiguous().clone()
               for g in (gu, gv, gw)]
        gabc = [torch.empty_like(ref) for _ in range(3)]
        work = torch.empty(max(1, fctx.every - 1) * gg.state_bytes(), dtype=torch.uint8, device=ref.device)
        gp = gg.adjoint_run(fctx.dt, fctx.nsteps, fctx.every, fctx.ckpt, work, lam, gabc)
        g1, g2, gt = gg.eig_backward(l1, l2, th, *gabc)
        gparams = torch.tensor(gp, dtype=params.dtype, device=params.device)
        fctx.ckpt = None
        return gparams, g1, g2, gt, lam[0], lam[1], lam[2], None, None, None, None


def default_every(nsteps: int) -> int:
    return max(1, int(math.ceil(math.sqrt(nsteps))))


def run(gg, params, lam1, lam2, theta, u0, v0, w0, dt, nsteps, every=None):
    """Differentiable nsteps-step run on the context ``gg`` (see module docstring)."""
    if every is None:
        every = default_every(nsteps)
    return FVRun.apply(params, lam1, lam2, theta, u0, v0, w0, gg, float(dt), int(nsteps), int(every))


def mismatch_loss(v, w, v_target, w_target, dx, dy):
    """Front-mismatch loss: one half of the area-weighted squared L2 distance of
    the tumour and acid fields from their targets."""
    return 0.5 * dx * dy * (((v - v_target) ** 2).sum() + ((w - w_target) ** 2).sum())
