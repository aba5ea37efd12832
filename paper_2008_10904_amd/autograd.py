"""torch.autograd face of the time-stepped resolvent: u_hat = R_d(mu) f_hat as a differentiable function of the
forcing coefficients and of a real reaction field mu added to the operator's diagonal.

The backward pass is the library's exact discrete adjoint of the RK4 march (resolvent_apply_backward), so the
gradients are those of the time-stepped map itself (what finite differences of the same run give), not of the
continuous resolvent.  With f_hat detached and set to the leading force modes, J = sum_j c_j ||u_hat_j|| has the
gradient of sum_j c_j sigma_1(w_j) with respect to mu, the leading mode being stationary (envelope argument).
"""
import numpy as np
import torch


class ResolventApply(torch.autograd.Function):
    """u_hat = ResolventApply.apply(f_hat, mu, op, grid, run, base_diag, checkpoint_every).

    f_hat: CUDA tensor [n_omega, k, N] of op's I/O dtype.  mu: real tensor [op.diag_size()] (any device) added to
    base_diag (complex [N] for a tridiagonal operator, real dfield [nz*ny*nx] for a grid operator); the operator's
    diagonal is set to base_diag + mu before the run."""

    @staticmethod
    def forward(ctx, f_hat, mu, op, grid, run, base_diag, checkpoint_every=0):
        _set(op, base_diag, mu)
        u_hat = op.apply(f_hat.contiguous(), grid, run)
        ctx.save_for_backward(f_hat, mu)
        ctx.op, ctx.grid, ctx.run, ctx.base, ctx.ckpt = op, grid, run, base_diag, checkpoint_every
        return u_hat

    @staticmethod
    def backward(ctx, g_hat):
        f_hat, mu = ctx.saved_tensors
        op = ctx.op
        _set(op, ctx.base, mu)  # the handle may have been re-used since the forward pass
        want_f, want_mu = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        f_grad, mu_grad = op.apply_backward(f_hat.contiguous(), g_hat.contiguous(), ctx.grid, ctx.run,
                                            ctx.ckpt, want_f=want_f, want_mu=want_mu)
        if mu_grad is not None:
            mu_grad = mu_grad.to(device=mu.device, dtype=mu.dtype)
        return f_grad, mu_grad, None, None, None, None, None


def _set(op, base_diag, mu):
    m = mu.detach().to("cpu", torch.float64).numpy().ravel()
    if m.size != op.diag_size():
        raise ValueError("mu has %d entries, the operator's diagonal %d" % (m.size, op.diag_size()))
    op.set_diagonal(np.asarray(base_diag) + m)


def resolvent_apply(f_hat, mu, op, grid, run, base_diag, checkpoint_every=0):
    """Functional form of ResolventApply."""
    return ResolventApply.apply(f_hat, mu, op, grid, run, base_diag, checkpoint_every)
