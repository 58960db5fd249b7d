"""torch.autograd.Function wrappers around the hand-written adjoints.

RasterizeFn: flat params -> field [C, H, W] complex64; backward calls
cgh_rasterize_adjoint, which recomputes each pixel's Gaussian response from the
per-tile lists instead of storing it.  The lists live in the context and are
replaced by every later rasterize on it; the forward records the context's
list generation, and a backward that finds another generation current first
rebuilds the lists of its own parameters (cgh_rasterize_lists: preprocess and
binning of Alg. 2, no per-pixel work), so interleaved forwards stay correct.
PropagateFn: field -> intensity [L, C, H, W]; backward calls
cgh_propagate_adjoint (conjugate transfer function, same band limit), which
recomputes the propagated field instead of storing it.
Gradients follow PyTorch's convention for complex tensors: dL/dRe + j dL/dIm.
"""
import torch


class RasterizeFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, params, cgh_ctx, n):
        params = params.contiguous()
        field = cgh_ctx.rasterize(params, n)
        ctx.cgh_ctx = cgh_ctx
        ctx.n = n
        ctx.generation = cgh_ctx.generation()
        ctx.save_for_backward(params)
        return field

    @staticmethod
    def backward(ctx, grad_field):
        (params,) = ctx.saved_tensors
        c = ctx.cgh_ctx
        if c.generation() != ctx.generation:
            c.rasterize_lists(params, ctx.n)
            ctx.generation = c.generation()
        grads = c.rasterize_adjoint(params, ctx.n, grad_field.contiguous())
        return grads, None, None


class PropagateFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, field, cgh_ctx):
        I, _ = cgh_ctx.propagate(field.contiguous())
        ctx.cgh_ctx = cgh_ctx
        ctx.save_for_backward(field)
        return I

    @staticmethod
    def backward(ctx, grad_intensity):
        (field,) = ctx.saved_tensors
        g = ctx.cgh_ctx.propagate_adjoint(field.contiguous(), grad_intensity.contiguous())
        return g, None


def rasterize(params, cgh_ctx, n):
    return RasterizeFn.apply(params, cgh_ctx, n)


def propagate(field, cgh_ctx):
    return PropagateFn.apply(field, cgh_ctx)
