"""Differentiable completion: K unrolled iterations of the HIP library as a
torch.autograd.Function (reverse mode, with checkpointing).

Forward: a completion at weights theta = (mu, rho1, rho2) runs K iterations from the real
initial factors (X0, Y0) and returns the completed tensor W^K; the iterate is saved
(tctf_get_state) every ``checkpoint_every`` iterations.  Backward: for each segment between
two checkpoints, from the last segment to the first, the segment's first checkpoint is
restored, the segment's iterations are run again keeping each iterate, and the library's
reverse pass of one iteration (tctf_adjoint_step) runs from the segment's last iteration
to its first; the adjoint of the set-up transforms (tctf_adjoint_initial) then gives the
gradients with respect to X0 and Y0.  Every arithmetic step of the backward pass runs in
the library's kernels: this module only sequences the calls and holds device buffers.
"""
from __future__ import annotations

import torch

from .binding import Completion, tctf_adjoint_initial, tctf_adjoint_step


class UnrolledCompletion(torch.autograd.Function):
    """W^K = unrolled(theta, X0, Y0; G, Omega, r, K).  theta: tensor (mu, rho1, rho2)."""

    @staticmethod
    def forward(ctx, theta, X0, Y0, G, omega, r, iters, checkpoint_every, eta):
        mu, rho1, rho2 = (float(v) for v in theta.detach().cpu().tolist())
        c = Completion(G, omega, r, mu=mu, rho1=rho1, rho2=rho2, eta=eta, X0=X0.detach().float(),
                       Y0=Y0.detach().float())
        ckpts = {0: c.get_state()}
        done = 0
        while done < iters:
            k = min(checkpoint_every, iters - done)
            c.step(k)
            done += k
            ckpts[done] = c.get_state()
        W = c.result()["W"]
        ctx.completion = c
        ctx.ckpts = ckpts
        ctx.theta_meta = (theta.device, theta.dtype)
        ctx.x_meta = (X0.device, X0.dtype)
        ctx.y_meta = (Y0.device, Y0.dtype)
        return W.to(torch.float64)

    @staticmethod
    def backward(ctx, W_bar):
        c = ctx.completion
        n1, n2, n3 = c.shape
        r = c.r
        nb = n3 // 2 + 1
        dev = c.G.device
        xt_bar = torch.zeros(nb * r * n1 * 2, dtype=torch.float64, device=dev)
        yt_bar = torch.zeros(nb * r * n2 * 2, dtype=torch.float64, device=dev)
        w_bar = W_bar.detach().to(device=dev, dtype=torch.float64).contiguous().clone()
        theta_bar = torch.zeros(3, dtype=torch.float64, device=dev)
        ws, nbytes = c.adjoint_workspace()
        bounds = sorted(ctx.ckpts)
        for a, b in reversed(list(zip(bounds[:-1], bounds[1:]))):
            c.set_state(ctx.ckpts[a])
            states = [ctx.ckpts[a]]
            for _ in range(a + 1, b):
                c.step(1)
                states.append(c.get_state())
            states.append(ctx.ckpts[b])
            for l in range(len(states) - 2, -1, -1):
                tctf_adjoint_step(c.ctx, states[l], states[l + 1], xt_bar, yt_bar, w_bar, theta_bar, ws, nbytes)
        x0_bar = torch.empty((n1, r, n3), dtype=torch.float64, device=dev)
        y0_bar = torch.empty((r, n2, n3), dtype=torch.float64, device=dev)
        tctf_adjoint_initial(c.ctx, xt_bar, yt_bar, x0_bar, y0_bar)
        c.close()
        ctx.completion = None
        return (theta_bar.to(*ctx.theta_meta), x0_bar.to(*ctx.x_meta), y0_bar.to(*ctx.y_meta),
                None, None, None, None, None, None)


def unrolled_completion(theta, X0, Y0, G, omega, r, iters, checkpoint_every=5, eta=1.0):
    """Completed tensor after ``iters`` iterations, differentiable with respect to theta =
    (mu, rho1, rho2), X0 and Y0 (FP32 forward, FP64 reverse pass)."""
    return UnrolledCompletion.apply(theta, X0, Y0, G, omega, r, iters, checkpoint_every, eta)


__all__ = ["UnrolledCompletion", "unrolled_completion"]
