"""torch.autograd front end of the hand-written adjoint.

`wperp(psi_e, make_sim, nsteps)` returns the transverse field energy
W = 1/2 sum (Ex^2 + Ey^2 + Bx^2 + By^2) dV after nsteps steps of a fresh
simulation built with correction coefficients psi_e (one row per instance),
as a differentiable function of psi_e.  The forward pass runs the GPU step
with checkpoints (pic_adjoint_forward); the backward pass runs the reverse
sweep with the adjoint kernels (pic_adjoint_backward) and scales the
gradient by the incoming cotangent.
"""
import numpy as np
import torch


class WperpFunction(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi_e, make_sim, nsteps):
        sim = make_sim(psi_e.detach().cpu().numpy().astype(np.float64))
        loss = sim.adjoint_forward(nsteps)
        ctx.sim = sim
        ctx.ncoef = psi_e.shape[-1]
        return torch.as_tensor(loss, dtype=psi_e.dtype)

    @staticmethod
    def backward(ctx, g):
        sim = ctx.sim
        grad = sim.adjoint_backward()[:, : ctx.ncoef]
        sim.close()
        ctx.sim = None
        gt = torch.as_tensor(grad, dtype=g.dtype)
        return g.reshape(-1, 1) * gt, None, None


def wperp(psi_e, make_sim, nsteps):
    """psi_e: tensor (n_inst, deg + 1); make_sim(psi_e ndarray) -> Simulation with
    adjoint_steps >= nsteps.  Returns W per instance (tensor, differentiable)."""
    return WperpFunction.apply(psi_e, make_sim, nsteps)
