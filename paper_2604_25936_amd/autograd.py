"""torch.autograd binding of the query path.

``sdf(model, dmap, xyz, ...)`` returns the signed distances as a tensor that
is differentiable with respect to ``xyz``: its backward calls
``sand_query_grad`` (the hand-written adjoint kernel), holding each point's
exit depth fixed as the forward found it. The depth map is piecewise
constant, so this is the derivative of the network the point actually ran
through.
"""

import torch

from . import sand


class SandSDF(torch.autograd.Function):
    @staticmethod
    def forward(ctx, xyz, model, dmap, precision, mode, max_depth):
        xyz = xyz.contiguous()
        depth = None
        if mode != "full":
            depth = torch.empty(xyz.shape[0], dtype=torch.uint8, device=xyz.device)
        y = sand.query(model, dmap, xyz, precision=precision, mode=mode, max_depth=max_depth,
                       depth_out=depth)
        ctx.save_for_backward(xyz, depth if depth is not None else torch.empty(0))
        ctx.model, ctx.dmap, ctx.precision, ctx.mode = model, dmap, precision, mode
        ctx.max_depth = max_depth
        return y

    @staticmethod
    def backward(ctx, dy):
        xyz, depth = ctx.saved_tensors
        if ctx.mode == "full":
            g = sand.query_grad(ctx.model, None, xyz, dy=dy.contiguous(), precision=ctx.precision,
                                mode="full", max_depth=ctx.max_depth)
        else:
            # replay the exit depths the forward used
            g = sand.query_grad(ctx.model, ctx.dmap, xyz, dy=dy.contiguous(),
                                precision=ctx.precision, mode="forced", forced_depth=depth)
        return g, None, None, None, None, None


def sdf(model, dmap, xyz, precision="fp32", mode="adaptive", max_depth=0):
    """Differentiable signed distances of float32 points [n, 3] on the GPU."""
    return SandSDF.apply(xyz, model, dmap, precision, mode, max_depth)
