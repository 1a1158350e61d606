"""Differentiable Jacobi sweeps (torch.autograd.Function wrappers).

The T-sweep operator is linear in (interior, shell): level s is
x_s = M x_{s-1} + G g, and the shell of every level equals g.  Its exact
adjoint therefore needs no forward state: the backward pass runs the
library's adjoint kernel (jacobi_adjoint), which sweeps lambda backwards and
accumulates the shell gradient.

JacobiT.apply(u, T, depth=None)   -> level T (grid with shell), differentiable
                                     in u; depth = sweeps fused per pass in both
                                     directions (None: library choice).
checkpoints(u, T, every, depth=None)
                                  -> levels every, 2*every, ..., T (the last
                                     may be shorter), each differentiable.  The
                                     forward keeps those levels; the backward
                                     runs one adjoint segment per interval and
                                     adds the gradient arriving at a checkpoint
                                     when it reaches that level (in the
                                     library), so losses on intermediate
                                     levels work.
"""
import torch

from . import jacobi


def _sweep(u, T, depth):
    a = u.detach().clone(memory_format=torch.contiguous_format)
    b = torch.empty_like(a)
    return jacobi.tblock(a, b, T, t=depth)


def _adjoint(grad, T, depth):
    lam_a = grad.detach().clone(memory_format=torch.contiguous_format)
    lam_b = torch.empty_like(lam_a)
    return jacobi.adjoint(lam_a, lam_b, T, t=depth)


class JacobiT(torch.autograd.Function):
    """Level T of the Jacobi iteration started from the grid u (interior =
    initial values, shell = Dirichlet data)."""

    @staticmethod
    def forward(ctx, u, T, depth=None):
        ctx.T, ctx.depth = int(T), depth
        return _sweep(u, int(T), depth)

    @staticmethod
    def backward(ctx, grad):
        if grad is None:
            return None, None, None
        return _adjoint(grad, ctx.T, ctx.depth), None, None


class _Checkpoints(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, T, every, depth):
        T, every = int(T), int(every)
        ctx.segments = []
        ctx.depth = depth
        outs = []
        cur = u.detach()
        done = 0
        while done < T:
            d = min(every, T - done)
            cur = _sweep(cur, d, depth)
            outs.append(cur)
            ctx.segments.append(d)
            done += d
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grads):
        lam = None
        for g, d in zip(reversed(grads), reversed(ctx.segments)):
            if g is not None:
                if lam is None:
                    lam = g.detach().clone(memory_format=torch.contiguous_format)
                else:
                    lam = jacobi.grid_add(lam, g.detach().contiguous())
            if lam is not None:
                lam = _adjoint(lam, d, ctx.depth)
        return lam, None, None, None


def checkpoints(u, T, every, depth=None):
    """Levels every, 2*every, ..., T of the iteration from u (a tuple)."""
    if T <= 0:
        return ()
    return _Checkpoints.apply(u, T, every, depth)
