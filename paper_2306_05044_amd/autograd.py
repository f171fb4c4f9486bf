"""Differentiable directional albedo: a torch.autograd.Function over the
estimator of Appendix A (L == 1) and its pathwise adjoint.

A cell's albedo depends only on that cell's parameters, so the Jacobian is
diagonal: three numbers per cell.  When any input needs a gradient, forward
runs ``albedo_value_and_grad``, which produces the value and those three
derivatives in one pass over the samples, and backward scales them by the
incoming gradient.  Otherwise forward runs the value-only kernel.  Nothing
but the inputs' derivatives is saved (no samples).
"""

from __future__ import annotations

import torch


class AlbedoFunction(torch.autograd.Function):
    """A(alpha_x, alpha_y, theta_o; phi_o, F0) per cell.

    Inputs: ax, ay, theta_o, phi_o, f0 -- float32 GPU tensors of one shape --
    then nsamples (int) and seed (int).  Gradients flow to ax, ay and theta_o
    (theta_o is the polar angle of the view direction, phi_o its azimuth) by
    the pathwise adjoint, and to f0 exactly (A is linear in F0); phi_o gets
    none.
    """

    @staticmethod
    def forward(ctx, ax, ay, theta_o, phi_o, f0, nsamples, seed):
        from . import albedo_estimate, albedo_value_and_grad
        # view direction from its spherical angles (argument marshalling)
        st = torch.sin(theta_o)
        wox = (st * torch.cos(phi_o)).contiguous().reshape(-1)
        woy = (st * torch.sin(phi_o)).contiguous().reshape(-1)
        woz = torch.cos(theta_o).contiguous().reshape(-1)
        axf, ayf = ax.contiguous().reshape(-1), ay.contiguous().reshape(-1)
        need = any(ctx.needs_input_grad[:3])
        a, gx, gy, gt = albedo_value_and_grad(
            wox, woy, woz, axf, ayf, int(nsamples), int(seed), f0=f0.contiguous().reshape(-1),
            with_grad=need)
        shape = ax.shape
        saved = [gx.reshape(shape), gy.reshape(shape), gt.reshape(shape)] if need else [None] * 3
        if ctx.needs_input_grad[4]:
            # the estimate is linear in F0: dA/dF0 = S1 - S5 on the same stream
            s1, s5 = albedo_estimate(wox, woy, woz, axf, ayf, int(nsamples), int(seed))
            saved.append((s1 - s5).reshape(shape))
        else:
            saved.append(None)
        ctx.save_for_backward(*saved)
        return a.reshape(shape)

    @staticmethod
    def backward(ctx, grad_a):
        jx, jy, jt, jf = ctx.saved_tensors
        g = grad_a.to(torch.float32)
        need = ctx.needs_input_grad
        return (g * jx if need[0] else None, g * jy if need[1] else None,
                g * jt if need[2] else None, None, g * jf if need[4] else None, None, None)


def albedo(ax, ay, theta_o, phi_o, f0, nsamples, seed):
    """Differentiable directional albedo (see AlbedoFunction)."""
    return AlbedoFunction.apply(ax, ay, theta_o, phi_o, f0, nsamples, seed)
