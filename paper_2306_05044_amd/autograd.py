"""Differentiable directional albedo: a torch.autograd.Function over the
estimator of Appendix A (L == 1) and its pathwise adjoint.

Forward runs ``albedo_estimate`` (both Fresnel sums from one stream) and
combines them for the per-cell F0; backward runs ``albedo_estimate_backward``,
which recomputes every sample from its Philox counter (no samples are saved,
only the inputs and the seed).
"""

from __future__ import annotations

import torch


class AlbedoFunction(torch.autograd.Function):
    """A(alpha_x, alpha_y, theta_o; phi_o, F0) per cell.

    Inputs: ax, ay, theta_o, phi_o, f0 -- float32 GPU tensors of one shape --
    then nsamples (int) and seed (int).  Gradients flow to ax, ay and theta_o
    (theta_o is the polar angle of the view direction, phi_o its azimuth).
    """

    @staticmethod
    def forward(ctx, ax, ay, theta_o, phi_o, f0, nsamples, seed):
        from . import albedo_estimate
        # view direction from its spherical angles (argument marshalling)
        st = torch.sin(theta_o)
        wox = (st * torch.cos(phi_o)).contiguous()
        woy = (st * torch.sin(phi_o)).contiguous()
        woz = torch.cos(theta_o).contiguous()
        axc, ayc, f0c = ax.contiguous(), ay.contiguous(), f0.contiguous()
        s1, s5 = albedo_estimate(wox.reshape(-1), woy.reshape(-1), woz.reshape(-1),
                                 axc.reshape(-1), ayc.reshape(-1), int(nsamples), int(seed))
        f = f0c.reshape(-1)
        a = f * s1 + (1.0 - f) * s5
        ctx.save_for_backward(wox, woy, woz, axc, ayc, f0c)
        ctx.nsamples = int(nsamples)
        ctx.seed = int(seed)
        return a.reshape(ax.shape)

    @staticmethod
    def backward(ctx, grad_a):
        from . import albedo_estimate_backward
        wox, woy, woz, ax, ay, f0 = ctx.saved_tensors
        g = grad_a.contiguous().reshape(-1).to(torch.float32)
        gx, gy, gt = albedo_estimate_backward(
            wox.reshape(-1), woy.reshape(-1), woz.reshape(-1), ax.reshape(-1), ay.reshape(-1),
            ctx.nsamples, ctx.seed, f0=f0.reshape(-1), grad_albedo=g)
        shape = ax.shape
        return (gx.reshape(shape), gy.reshape(shape), gt.reshape(shape), None, None, None, None)


def albedo(ax, ay, theta_o, phi_o, f0, nsamples, seed):
    """Differentiable directional albedo (see AlbedoFunction)."""
    return AlbedoFunction.apply(ax, ay, theta_o, phi_o, f0, nsamples, seed)
