"""torch.autograd wrapper of the library's differentiable rollout.

Marshalling only: the forward steps, the checkpoints, the recomputation and
the adjoint sweeps all run in libjgs2 (jgs2_rollout, jgs2_rollout_backward).
"""
import numpy as np
import torch


class Simulate(torch.autograd.Function):
    """x_N = Simulate.apply(log_E, u, solver, nu, rho, n_steps, ckpt_every)

    Runs n_steps implicit-Euler steps of ``solver``'s mesh from its rest
    shape, with per-tet Young's modulus exp(log_E) and the initial velocity u
    (3,) on every free vertex, and returns the final positions (nV, 3).
    Gradients flow to log_E (nT,) and u (3,)."""

    @staticmethod
    def forward(ctx, log_E, u, solver, nu, rho, n_steps, ckpt_every):
        solver.set_material_log_e(log_E.detach().cpu().double().numpy(), nu, rho)
        v0 = np.zeros((solver.nV, 3))
        v0[~solver.pinned] = u.detach().cpu().double().numpy()[None, :]
        solver.set_state(solver.X, v0)
        solver.rollout(int(n_steps), int(ckpt_every))
        x, _ = solver.get_state()
        ctx.solver = solver
        ctx.dev = log_E.device
        return torch.from_numpy(x).to(ctx.dev)

    @staticmethod
    def backward(ctx, gx):
        s = ctx.solver
        th, _, _, stats = s.rollout_backward(gx.detach().cpu().double().numpy())
        ctx.stats = stats
        return (torch.from_numpy(th).to(ctx.dev), torch.from_numpy(stats["ubar"]).to(ctx.dev),
                None, None, None, None, None)
