"""torch.autograd.Function over the fused forward and adjoint kernels.

The forward pass returns per-pixel estimates I_p(theta) of the Gaussian-lobe integrand; the
backward pass calls the adjoint kernel, which recomputes the samples from their indices and
returns dL/dtheta = sum_p dL/dI_p (1/N_p) sum_i df(x_pi)/dtheta.  Only the lobe parameters
theta are differentiable.
"""

import torch


class QMCIntegrate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, sampler, integrand, width, height, counts):
        from . import qmc_integrate_pixels

        ig = integrand.with_params(theta.detach().contiguous())
        means = qmc_integrate_pixels(sampler, ig, width, height, counts)
        ctx.sampler, ctx.integrand, ctx.shape = sampler, ig, (width, height)
        ctx.save_for_backward(counts)
        ctx.theta_shape = theta.shape
        return means

    @staticmethod
    def backward(ctx, grad_means):
        from . import qmc_integrate_pixels_backward

        (counts,) = ctx.saved_tensors
        width, height = ctx.shape
        g = qmc_integrate_pixels_backward(ctx.sampler, ctx.integrand, width, height, counts,
                                          grad_means.contiguous().float())
        return g.view(ctx.theta_shape), None, None, None, None, None


def integrate(theta, sampler, integrand, width, height, counts):
    """Differentiable per-pixel estimates (float32 [width*height])."""
    return QMCIntegrate.apply(theta, sampler, integrand, width, height, counts)
