"""torch.autograd.Function around tem_forward / tem_adjoint (Sec. 4).

    d = receiver_data(log_sigma, ctx, loops, receivers, xi, c)
    loss = f(d); loss.backward()        # log_sigma.grad = J^T (dloss/dd)

The forward runs tem_forward with the solutions kept on the device; the
backward hands dloss/dd to tem_adjoint, which solves the J adjoint shifted
systems with the stored forward solutions and returns dloss/d ln sigma per
cell.  Both directions run in libtem.so; this module only moves tensors.
"""
from __future__ import annotations

import numpy as np
import torch


class ReceiverData(torch.autograd.Function):
    @staticmethod
    def forward(fctx, log_sigma, ctx, loops, receivers, xi, c, opts):
        opts = dict(opts)
        # recompute=True keeps no forward solutions on the device: the backward
        # solves for them again (one more multi-shift solve per source)
        keep = not opts.pop("recompute", False)
        ctx.set_conductivity(log_sigma.detach(), log=True)
        data, _ = ctx.forward(loops, receivers, xi, c, keep_solutions=keep, **opts)
        fctx.tem_ctx = ctx
        fctx.generation = ctx.generation
        fctx.sigma_shape = log_sigma.shape
        fctx.device = log_sigma.device
        return torch.from_numpy(data).to(log_sigma.device, torch.float64)

    @staticmethod
    def backward(fctx, grad_data):
        ctx = fctx.tem_ctx
        # the adjoint reuses the solutions stored by this forward: any later
        # forward or conductivity change on the context has replaced them
        if ctx.generation != fctx.generation:
            raise RuntimeError("the context ran another forward or conductivity update after this one; "
                               "use one context per differentiated model")
        w = grad_data.detach().to("cpu", torch.float64).numpy()
        grad, _ = ctx.adjoint(np.ascontiguousarray(w))
        g = torch.from_numpy(grad).to(fctx.device, torch.float64)
        return g.reshape(fctx.sigma_shape), None, None, None, None, None, None


def receiver_data(log_sigma, ctx, loops, receivers, xi, c, **opts):
    """dB_z/dt data (n_src, T, n_rx) of the model ln sigma (nz, ny, nx), with a
    gradient w.r.t. ln sigma through the adjoint solves.  opts go to
    Context.forward; recompute=True trades memory for one more solve per
    source in the backward."""
    return ReceiverData.apply(log_sigma, ctx, loops, receivers, xi, c, opts)
