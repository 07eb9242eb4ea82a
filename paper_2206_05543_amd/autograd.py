"""torch.autograd wrapper of k V(1,1) cycles: u_K = V^K(u_0, b; c).

The forward pass runs the library's FP64 cycles and keeps one checkpoint of
the iterate per cycle; the backward pass calls the hand-written adjoint cycle
(mg_vcycle_adjoint) once per cycle in reverse order, recomputing every
level's states from the checkpoint.  Gradients flow to the smoother
coefficients c (any float dtype; promoted to FP64 for the cycle, gradient
accumulated in FP64), to b and to u_0.

Checkpoints are written by the library (mg_checkpoint) and read by it
(mg_vcycle_adjoint).  With checkpoint_dtype=torch.float32 the forward pass
rounds each cycle-start iterate to FP32, stores it, and continues from the
rounded value, so the backward recomputation reproduces the forward states
bit for bit.  The rounding itself is piecewise constant; the backward pass
treats it as the identity (a straight-through derivative).  For K >= 2 the
gradient is therefore that of the FP64 cycles evaluated on the rounded
states, which differs from the gradient of the unrounded FP64 map by
O(2^-24) relative.
"""
import math

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
            ck = torch.empty(u.shape, dtype=ckpt_dtype, device=u.device)
            mg.checkpoint(u, ck)  # FP32: u becomes the rounded value
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
            cbar = mg.vcycle_adjoint(ctx.b64, ck, ubar, ubar, bbar, cbar)
        dt, dev = ctx.coeff_meta
        gc = torch.tensor(cbar, dtype=torch.float64).to(dtype=dt, device=dev)
        return gc, bbar, ubar, None, None, None


def kcycles(mg: Multigrid, coeffs, b, u0, K, checkpoint_dtype=torch.float64):
    """u_K after K V(1,1) cycles from u0 with smoother coefficients `coeffs`
    (1-D tensor of 3 (2D) or 2 (3D) values), differentiable in coeffs, b and
    u0.  b and u0 are CUDA tensors with mg.batch * (N-1)^d elements."""
    return _KCycles.apply(coeffs, b, u0, mg, int(K), checkpoint_dtype)


def descend(mg: Multigrid, coeffs, e0, b, K, max_iter=200, rtol=1e-7,
            checkpoint_dtype=torch.float32, armijo=1e-4):
    """Plain gradient descent with Armijo backtracking, in FP64, on the
    smoother coefficients for the k-cycle loss L(c) = sum over the batch of
    ||V^K(e0, b; c)||^2, with gradients from the adjoint cycle.

    The first step moves the coefficients by 1% of their norm; after an
    accepted step the trial step doubles, and it halves until the Armijo
    condition L(c - a g) <= L(c) - armijo a |g|^2 holds.  Stops when the
    accepted step is below rtol |c| or after max_iter steps.  Returns a dict
    with the final coefficients, loss, gradient and the loss history."""
    c = torch.as_tensor(coeffs, dtype=torch.float64).detach().clone().cpu()

    def loss(cc, grad):
        cp = cc.clone().requires_grad_(grad)
        u = kcycles(mg, cp, b, e0, K, checkpoint_dtype)
        L = (u * u).sum()
        if not grad:
            return float(L), None
        L.backward()
        return float(L), cp.grad.detach().clone()

    L, g = loss(c, True)
    hist = [L]
    alpha = None
    it = 0
    for it in range(1, max_iter + 1):
        gn = float(g.norm())
        if gn == 0.0:
            break
        alpha = 1e-2 * float(c.norm()) / gn if alpha is None else 2.0 * alpha
        while True:
            cn = c - alpha * g
            Ln, _ = loss(cn, False)
            if Ln <= L - armijo * alpha * gn * gn:
                break
            alpha *= 0.5
            if alpha * gn <= 1e-16 * float(c.norm()):
                break
        step = alpha * gn
        if Ln > L:  # no descent possible at working precision
            break
        c = cn
        L, g = loss(c, True)
        hist.append(L)
        if step <= rtol * float(c.norm()):
            break
    return {"coeffs": c.tolist(), "loss": L, "grad": g.tolist(), "iterations": it,
            "history": hist}
