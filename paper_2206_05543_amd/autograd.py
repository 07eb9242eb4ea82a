"""torch.autograd wrapper of k V(1,1) cycles: u_K = V^K(u_0, b; c).

The forward pass runs the library's FP64 cycles and keeps one checkpoint of
the iterate per cycle; the backward pass calls the hand-written adjoint cycle
(mg_vcycle_adjoint) once per cycle in reverse order, recomputing every
level's states from the checkpoint.  Gradients flow to the smoother
coefficients c (any float dtype; promoted to FP64 for the cycle, gradient
accumulated in FP64), to b and to u_0.

With checkpoint_dtype=torch.float32 the forward pass rounds each cycle-start
iterate to FP32, stores it, and continues from the rounded value; the
recomputation in the backward pass is then bit-identical to the forward pass
and the gradient is exact for the computed forward map.
"""
import torch

from ._lib import Multigrid


class _KCycles(torch.autograd.Function):
    @staticmethod
    def forward(ctx, coeffs, b, u0, mg, K, ckpt_dtype):
        c = [float(x) for x in coeffs.detach().double().cpu().tolist()]
        mg.set_coeffs(c)
        b64 = b.detach().to(torch.float64).contiguous()
        u = u0.detach().to(torch.float64).contiguous().clone()
        ckpts = []
        for _ in range(K):
            if ckpt_dtype == torch.float64:
                ckpts.append(u.clone())
            else:
                ck = u.to(ckpt_dtype)
                u = ck.to(torch.float64).contiguous()
                ckpts.append(ck)
            mg.vcycle(b64, u)
        ctx.mg, ctx.c, ctx.b64, ctx.ckpts = mg, c, b64, ckpts
        ctx.coeff_meta = (coeffs.dtype, coeffs.device)
        return u

    @staticmethod
    def backward(ctx, gu):
        mg = ctx.mg
        mg.set_coeffs(ctx.c)
        ubar = gu.detach().to(torch.float64).contiguous().clone()
        bbar = torch.zeros_like(ctx.b64)
        cbar = [0.0] * len(ctx.c)
        for ck in reversed(ctx.ckpts):
            uin = ck.to(torch.float64).contiguous()
            cbar = mg.vcycle_adjoint(ctx.b64, uin, ubar, ubar, bbar, cbar)
        dt, dev = ctx.coeff_meta
        gc = torch.tensor(cbar, dtype=torch.float64).to(dtype=dt, device=dev)
        return gc, bbar, ubar, None, None, None


def kcycles(mg: Multigrid, coeffs, b, u0, K, checkpoint_dtype=torch.float64):
    """u_K after K V(1,1) cycles from u0 with smoother coefficients `coeffs`
    (1-D tensor of 3 (2D) or 2 (3D) values), differentiable in coeffs, b and
    u0.  b and u0 are CUDA tensors with mg.batch * (N-1)^d elements."""
    return _KCycles.apply(coeffs, b, u0, mg, int(K), checkpoint_dtype)
