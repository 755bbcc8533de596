"""Psi(q) as a differentiable torch function backed by the library's kernels.

    psi = hamlet_logpost(plan, q_modes, q_dist, q_snl)
    psi.backward()      # q_modes.grad, q_dist.grad, q_snl.grad

The forward pass runs one log-posterior-and-gradient evaluation
(hamlet_logpost_grad_entries: three inverse FFTs with the CIC gather, the
likelihood, the CIC scatter and three forward FFTs with the adjoint
multiply) and keeps the gradient; backward scales it by the incoming
gradient.  Mode gradients follow torch's convention for real functions of
complex tensors, dPsi/dRe + i dPsi/dIm per stored entry (each member of a
Hermitian pair on the kz = 0 plane is its own variable there).
"""
import torch

from . import hamlet


class LogPosterior(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q_modes, q_dist, q_snl, plan):
        g = plan.zeros_modes()
        gd = plan.zeros_dist()
        gs = plan.scalar()
        psi = plan.scalar()
        hamlet.logpost_grad([plan], [q_modes.detach().contiguous()], [q_dist.detach().contiguous()],
                            [q_snl.detach().contiguous()], [g], [gd], [gs], [psi], per_entry=True)
        ctx.save_for_backward(g, gd, gs)
        return psi.reshape(())

    @staticmethod
    def backward(ctx, grad_out):
        g, gd, gs = ctx.saved_tensors
        return grad_out * g, grad_out * gd, grad_out * gs, None


def hamlet_logpost(plan, q_modes, q_dist, q_snl):
    """Psi = -ln Pi(q) (a 0-d float64 tensor) with gradients to the inputs."""
    return LogPosterior.apply(q_modes, q_dist, q_snl, plan)
