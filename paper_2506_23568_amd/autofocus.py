"""Trajectory autofocus: gradient steps on a smooth motion-error model of the
antenna positions through the library's forward, loss and backward kernels.

Each step images the echoes at the current positions (hhffbp_image, frozen
plan), forms the entropy + relative-L2 loss and its cotangent
(hhffbp_image_stats, hhffbp_loss_grad), pulls the cotangent back to the
positions (hhffbp_backward, position gradient only), maps it onto the model's
coefficients and applies one Adam update (torch.optim, on the device).
Handheld motion errors that the positioning system leaves in the trajectory
blur the image (Sec. I names autofocus as the usual remedy); the backward
kernels make that correction a gradient method.

Motion model: positions = p0 + B c, with B the first K cosine modes over the
acquisition index, cos(pi m (i + 1/2) / N) for m = 0..K-1, one coefficient
column per axis.  Free per-position updates (K = 0) are available too.

Objective: by default the relative L2 distance to a reference image of the
same scene (the clean-trajectory image).  The image entropy is available as a
second term; on scenes dominated by distributed random reflectivity, lowering
it does not lead towards the true trajectory.
"""
import math

import torch

from .binding import HHFFBPError, image_stats, loss_grad


def cosine_basis(n, k, device):
    """[n, k] float64: column m is cos(pi m (i + 1/2) / n) over the index i."""
    t = (torch.arange(n, dtype=torch.float64, device=device) + 0.5) * (math.pi / n)
    return torch.cos(t[:, None] * torch.arange(k, dtype=torch.float64, device=device)[None, :])


def autofocus(plan, echoes, positions, steps=20, lr=3e-5, clean=None, modes=16, w_entropy=0.0,
              w_l2=1.0, on_step=None):
    """Run ``steps`` Adam steps (learning rate ``lr`` metres) on the motion model
    around ``positions`` (float64 [n_pos, 3] on the plan's device).

    ``modes``: cosine modes per axis (0 = every coordinate free).  The loss is
    w_entropy H(f) + w_l2 ||f - clean||^2 / ||clean||^2 (``clean`` an optional
    complex64 image; without it only the entropy term).  Returns (positions,
    history); history holds, per step, the loss before the update and the
    step's device time in ms (forward, loss, backward and update).
    ``on_step(k, positions, image)`` is called after each image, before the
    update, if given."""
    p0 = positions.detach().contiguous()
    dev = p0.device
    if modes > 0:
        B = cosine_basis(p0.shape[0], modes, dev)
        c = torch.zeros((modes, 3), dtype=torch.float64, device=dev, requires_grad=True)
    else:
        B = None
        c = torch.zeros_like(p0, requires_grad=True)
    opt = torch.optim.Adam([c], lr=lr)
    ws = plan._workspace(torch, backward=True)
    img = torch.empty(plan.dims, dtype=torch.complex64, device=dev)
    stream = torch.cuda.current_stream(dev)
    # the slack check runs on a stream of its own (default priority), so that
    # the host's wait for its count overlaps the image instead of stalling the GPU
    side = torch.cuda.Stream(device=dev)
    hist = []

    def current():
        return (p0 + (c.detach() if B is None else B @ c.detach())).contiguous()

    for k in range(steps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        pos = current()
        ready = torch.cuda.Event()
        ready.record(stream)
        plan.image(echoes, positions=pos, out=img, workspace=ws)
        # the plan's windows hold positions within its slack; beyond it the
        # kernels clamp, so stop rather than descend on clamped positions
        side.wait_event(ready)
        n_out = plan.check_positions(pos, stream=side.cuda_stream)
        if n_out:
            raise HHFFBPError(-1, f"autofocus step {k}: {n_out} positions moved beyond the plan's "
                                  f"slack of {plan.config.position_slack} m; plan again around "
                                  "the current positions")
        st = image_stats(img, clean)
        loss, g = loss_grad(img, clean, st, w_entropy=w_entropy, w_l2=w_l2)
        if on_step is not None:
            on_step(k, pos, img)
        _, gp = plan.backward(echoes, g, positions=pos, want_echoes=False, workspace=ws)
        # B^T gp as a reduction: the BLAS product of a 16 x N by N x 3 pair
        # runs on a single workgroup (~1.9 ms at N = 65536)
        c.grad = gp if B is None else (B[:, :, None] * gp[:, None, :]).sum(0)
        opt.step()
        e1.record(stream)
        torch.cuda.synchronize()
        hist.append({"loss": loss.item(), "ms": e0.elapsed_time(e1)})
    return current(), hist
