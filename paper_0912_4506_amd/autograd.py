"""Differentiable Jacobi sweeps (torch.autograd.Function wrappers).

The T-sweep operator is linear in (interior, shell): level s is
x_s = M x_{s-1} + G g, the shell of every level equals g.  Its exact adjoint
therefore needs no forward state; the backward pass runs the library's
adjoint kernel (jacobi_adjoint), which sweeps lambda backwards t levels per
pass and accumulates the shell gradient.

JacobiT.apply(u, T, t)        -> level T (grid with shell), differentiable in u.
checkpoints(u, T, t)          -> levels t, 2t, ..., T (the last may be shorter),
                                 each differentiable: gradients arriving at a
                                 checkpoint are added to lambda when the backward
                                 pass reaches that level.
"""
import torch

from . import jacobi


def _sweep(u, T, t):
    a = u.detach().clone(memory_format=torch.contiguous_format)
    b = torch.empty_like(a)
    return jacobi.tblock(a, b, T, t=t)


def _adjoint(grad, T, t):
    lam_a = grad.detach().clone(memory_format=torch.contiguous_format)
    lam_b = torch.empty_like(lam_a)
    return jacobi.adjoint(lam_a, lam_b, T, t=t)


class JacobiT(torch.autograd.Function):
    """Level T of the Jacobi iteration started from the grid u (interior =
    initial values, shell = Dirichlet data)."""

    @staticmethod
    def forward(ctx, u, T, t=None):
        ctx.T, ctx.t = int(T), t
        return _sweep(u, int(T), t)

    @staticmethod
    def backward(ctx, grad):
        if grad is None:
            return None, None, None
        return _adjoint(grad, ctx.T, ctx.t), None, None


class _Checkpoints(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, T, t):
        T, t = int(T), int(t)
        ctx.depths = []
        outs = []
        cur = u.detach()
        done = 0
        while done < T:
            d = min(t, T - done)
            cur = _sweep(cur, d, d)
            outs.append(cur)
            ctx.depths.append(d)
            done += d
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grads):
        lam = None
        for g, d in zip(reversed(grads), reversed(ctx.depths)):
            if g is not None:
                lam = g.clone() if lam is None else lam + g
            if lam is not None:
                lam = _adjoint(lam, d, d)
        return lam, None, None


def checkpoints(u, T, t):
    """Levels t, 2t, ..., T of the iteration from u (a tuple of grids)."""
    if T <= 0:
        return ()
    return _Checkpoints.apply(u, T, t)
