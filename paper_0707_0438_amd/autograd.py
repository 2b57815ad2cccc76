"""torch.autograd bindings of the library's forward and adjoint entry points.

Both functions only marshal tensors: the forward calls nbody_force /
nbody_shared_run and the backward calls nbody_force_vjp_self /
nbody_shared_adjoint (hand-written HIP adjoint kernels).

* :class:`NBodyForce` -- (acc, jerk, pot) of one self-gravitating set.
* :class:`HermiteShared` -- positions and velocities after ``nsteps`` shared
  Hermite steps, checkpointed every ``ckpt_every`` steps; the backward
  recomputes each segment from its checkpoint.
"""
from __future__ import annotations

import torch

from . import Context


class NBodyForce(torch.autograd.Function):
    """acc, jerk, pot = NBodyForce.apply(ctx, x, v, m, eps, G, prec);
    x, v: (3, n) float64 GPU tensors, m: (n,)."""

    @staticmethod
    def forward(fctx, ctx: Context, x, v, m, eps, G=1.0, prec="ds"):
        n = x.shape[1]
        idx = torch.arange(n, dtype=torch.int32, device=x.device)
        acc, jerk, pot = ctx.force(x.detach().contiguous(), v.detach().contiguous(),
                                   x.detach().contiguous(), v.detach().contiguous(),
                                   m.detach().contiguous(), eps, G=G, prec=prec, i_self=idx)
        fctx.save_for_backward(x, v, m)
        fctx.args = (ctx, eps, G, prec)
        return acc, jerk, pot

    @staticmethod
    def backward(fctx, ga, gj, gp):
        x, v, m = fctx.saved_tensors
        ctx, eps, G, prec = fctx.args
        zero3 = lambda: torch.zeros_like(x)
        ga = zero3() if ga is None else ga.contiguous()
        gj = None if gj is None else gj.contiguous()
        gp = None if gp is None else gp.contiguous()
        gx, gv, gm = ctx.force_vjp_self(x.detach().contiguous(), v.detach().contiguous(),
                                        m.detach().contiguous(), eps, ga, gj, gp, G=G, prec=prec)
        return None, gx, gv, gm, None, None, None


class HermiteShared(torch.autograd.Function):
    """x_T, v_T = HermiteShared.apply(ctx, x0, v0, m, eps, dt, nsteps, ckpt_every, G, prec)."""

    @staticmethod
    def forward(fctx, ctx: Context, x0, v0, m, eps, dt, nsteps, ckpt_every=8, G=1.0, prec="ds"):
        x0c, v0c, mc = x0.detach().contiguous(), v0.detach().contiguous(), m.detach().contiguous()
        xT, vT, ck = ctx.shared_run(x0c, v0c, mc, eps, dt, nsteps, G=G, prec=prec,
                                    ckpt_every=ckpt_every, checkpoints=True)
        fctx.save_for_backward(x0c, v0c, mc, ck)
        fctx.args = (ctx, eps, dt, nsteps, ckpt_every, G, prec)
        return xT, vT

    @staticmethod
    def backward(fctx, gxT, gvT):
        x0, v0, m, ck = fctx.saved_tensors
        ctx, eps, dt, nsteps, every, G, prec = fctx.args
        gxT = torch.zeros_like(x0) if gxT is None else gxT.contiguous()
        gvT = None if gvT is None else gvT.contiguous()
        gx0, gv0, gm = ctx.shared_adjoint(x0, v0, m, eps, dt, nsteps, ck, gxT, gvT, G=G, prec=prec,
                                          ckpt_every=every)
        return None, gx0, gv0, gm, None, None, None, None, None, None
