"""Differentiable wrappers around the HIP library.

``SRForce``: accelerations from positions, with a hand-written adjoint
(the library's VJP kernel); the backward pass reuses the forward's binning
while the library still holds it, and otherwise re-bins from the saved
float64 positions.

``SKSRollout``: n_c short-range subcycles of the symmetric stream-kick-stream
map (Habib et al. 2012, Sec. II, Eq. 6), x1 = x + h/2 v, v' = v + h a(x1),
x' = x1 + h/2 v'.  The forward pass checkpoints x1 of every subcycle (float64)
and nothing else; the backward pass walks the subcycles in reverse,
recomputing each force derivative at its checkpoint (the last subcycle's
VJP reuses the forward's binning when it is still in the workspace):
gv += h/2 gx;  gx += J(x1)^T (h gv);  gv += h/2 gx.
All arithmetic runs in the library's kernels; torch only allocates.
"""
from __future__ import annotations

import torch

from . import _lib


class SRForce(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos, mass, box, r_cut, eps, poly):
        acc = _lib.force(pos, mass, box, r_cut, eps, poly)
        ctx.save_for_backward(pos, mass)
        ctx.params = (box, r_cut, eps, poly)
        ctx.token = _lib.binning_token()
        return acc

    @staticmethod
    def backward(ctx, grad_acc):
        pos, mass = ctx.saved_tensors
        box, r_cut, eps, poly = ctx.params
        g = grad_acc.contiguous()
        if g.dtype != torch.float32:
            raise TypeError("cotangent of the accelerations must be float32")
        gpos = _lib.force_vjp(pos, mass, box, r_cut, eps, poly, g, binned=ctx.token)
        return gpos, None, None, None, None, None


def sr_force(pos, mass, box, r_cut, eps, poly):
    """Differentiable short-range accelerations (float32, input order)."""
    return SRForce.apply(pos, mass, box, r_cut, eps, poly)


def sks_forward(x, v, mass, box, r_cut, eps, poly, h, n_c, checkpoints=None):
    """Advance (x, v) in place by n_c subcycles; appends x1 copies to
    ``checkpoints`` when given.  Returns (x, v, token): the binning token of
    the last force call (its binning serves the first VJP of the reverse
    pass, at the same position, while it stays in the workspace)."""
    acc = torch.empty(x.shape, dtype=torch.float32, device=x.device)
    token = 0
    for _ in range(n_c):
        _lib.stream(x, v, 0.5 * h, box)
        if checkpoints is not None:
            checkpoints.append(x.clone())
        _lib.force(x, mass, box, r_cut, eps, poly, out=acc)
        token = _lib.binning_token()
        _lib.kick(v, acc, h)
        _lib.stream(x, v, 0.5 * h, box)
    return x, v, token


class SKSRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x0, v0, mass, box, r_cut, eps, poly, h, n_c):
        x = x0.detach().clone()
        v = v0.detach().clone()
        cps: list = []
        _, _, token = sks_forward(x, v, mass, box, r_cut, eps, poly, h, n_c, cps)
        ctx.save_for_backward(mass, *cps)
        ctx.params = (box, r_cut, eps, poly, h)
        ctx.token = token
        return x, v

    @staticmethod
    def backward(ctx, gx_out, gv_out):
        mass, *cps = ctx.saved_tensors
        box, r_cut, eps, poly, h = ctx.params
        x_like = cps[0]
        gx = (gx_out.detach().to(torch.float64).clone() if gx_out is not None
              else torch.zeros_like(x_like))
        gv = (gv_out.detach().to(torch.float64).clone() if gv_out is not None
              else torch.zeros_like(x_like))
        gx = gx.contiguous()
        gv = gv.contiguous()
        ga = torch.empty(x_like.shape, dtype=torch.float32, device=x_like.device)
        tmp = torch.empty_like(gx)
        token = ctx.token                              # binning of the last x1
        for x1 in reversed(cps):
            _lib.stream(gv, gx, 0.5 * h, 0.0)          # gv += h/2 gx
            _lib.kick_adjoint(gv, h, out=ga)           # ga = h gv
            _lib.force_vjp(x1, mass, box, r_cut, eps, poly, ga, out=tmp, binned=token)
            token = 0
            _lib.stream(gx, tmp, 1.0, 0.0)             # gx += J^T ga
            _lib.stream(gv, gx, 0.5 * h, 0.0)          # gv += h/2 gx
        return gx, gv, None, None, None, None, None, None, None


def rollout_sks(x0, v0, mass, box, r_cut, eps, poly, h, n_c):
    """Differentiable n_c-subcycle rollout; returns (x, v) after the steps."""
    return SKSRollout.apply(x0, v0, mass, box, r_cut, eps, poly, h, n_c)
