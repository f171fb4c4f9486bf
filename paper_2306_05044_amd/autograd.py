"""Differentiable directional albedo: a torch.autograd.Function over the
estimator of Appendix A (L == 1) and its pathwise adjoint.

A cell's albedo depends only on that cell's parameters, so the Jacobian is
diagonal: three numbers per cell.  When any input needs a gradient, forward
runs ``albedo_value_and_grad``, which produces the value and those three
derivatives in one pass over the samples, and backward scales them by the
incoming gradient (``albedo_apply_jacobian``).  Otherwise forward runs the
value-only kernel.  The view direction comes from its angles in
``albedo_view_from_angles``, so every arithmetic step runs in the library's
kernels.  Nothing but the inputs' derivatives is saved (no samples).
"""

from __future__ import annotations

import torch


class AlbedoFunction(torch.autograd.Function):
    """A(alpha_x, alpha_y, theta_o; phi_o, F0) per cell.

    Inputs: ax, ay, theta_o, phi_o, f0 -- float32 GPU tensors of one shape --
    then nsamples (an int for every cell, or an int64 tensor of that shape
    with each cell's count) and seed (int).  Gradients flow to ax, ay and theta_o
    (theta_o is the polar angle of the view direction, phi_o its azimuth) by
    the pathwise adjoint, and to f0 exactly (A is linear in F0); phi_o gets
    none.
    """

    @staticmethod
    def forward(ctx, ax, ay, theta_o, phi_o, f0, nsamples, seed):
        from . import albedo_estimate, albedo_value_and_grad, albedo_view_from_angles
        flat = [t.contiguous().reshape(-1) for t in (ax, ay, theta_o, phi_o, f0)]
        axf, ayf, thf, phf, f0f = flat
        ns = (nsamples.contiguous().reshape(-1) if isinstance(nsamples, torch.Tensor)
              else int(nsamples))
        wox, woy, woz = albedo_view_from_angles(thf, phf)
        need = any(ctx.needs_input_grad[:3])
        a, gx, gy, gt = albedo_value_and_grad(
            wox, woy, woz, axf, ayf, ns, int(seed), f0=f0f, with_grad=need)
        saved = [gx, gy, gt] if need else [None] * 3
        if ctx.needs_input_grad[4]:
            # the estimate is linear in F0: dA/dF0 = S1 - S5 on the same stream
            saved += list(albedo_estimate(wox, woy, woz, axf, ayf, ns, int(seed)))
        else:
            saved += [None, None]
        ctx.save_for_backward(*saved)
        ctx.shape = ax.shape
        return a.reshape(ax.shape)

    @staticmethod
    def backward(ctx, grad_a):
        from . import albedo_apply_jacobian
        jx, jy, jt, s1, s5 = ctx.saved_tensors
        need = ctx.needs_input_grad
        g = grad_a.to(torch.float32).contiguous().reshape(-1)
        ox, oy, ot, of = albedo_apply_jacobian(
            g, jx if need[0] else None, jy if need[1] else None, jt if need[2] else None,
            s1 if need[4] else None, s5 if need[4] else None)
        shape = ctx.shape

        def out(t):
            return None if t is None else t.reshape(shape)

        return out(ox), out(oy), out(ot), None, out(of), None, None


def albedo(ax, ay, theta_o, phi_o, f0, nsamples, seed):
    """Differentiable directional albedo (see AlbedoFunction)."""
    return AlbedoFunction.apply(ax, ay, theta_o, phi_o, f0, nsamples, seed)
