"""torch.autograd.Function over hhffbp_image / hhffbp_backward.

The forward and backward passes both run in the library's HIP kernels; this
module only hands tensors to them.  Gradients follow torch's convention for
complex tensors (dL/dRe + j dL/dIm); the plan stays frozen.
"""
import torch


class HHFFBPFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, echoes, positions, plan):
        img = plan.image(echoes, positions=positions)
        ctx.plan = plan
        ctx.save_for_backward(echoes, positions if positions is not None else torch.empty(0))
        ctx.has_positions = positions is not None
        return img

    @staticmethod
    def backward(ctx, grad_image):
        echoes, positions = ctx.saved_tensors
        positions = positions if ctx.has_positions else None
        want_s = ctx.needs_input_grad[0]
        want_p = ctx.needs_input_grad[1]
        if not (want_s or want_p):
            return None, None, None
        ge, gp = ctx.plan.backward(echoes, grad_image.to(torch.complex64).contiguous(),
                                   positions=positions, want_echoes=want_s,
                                   want_positions=want_p)
        return ge, gp, None


def hhffbp_image(echoes, positions, plan):
    """Differentiable image: echoes complex64 (n_pos, n_f), positions float64 (n_pos, 3) or None."""
    return HHFFBPFunction.apply(echoes, positions, plan)
