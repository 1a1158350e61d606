"""Mixed-precision Laplace solve: FP64 iterative refinement around FP32
temporally blocked Jacobi sweeps (a form added on top of the paper's method).

The system is the one whose fixed point the Jacobi update of Sect. 1.1 of the
paper seeks: A x = b with A = 6I - (interior adjacency) and b = the sum of
each cell's shell neighbours, i.e. r = b - A x = (six neighbours of x) - 6x
with the shell of x as Dirichlet data.

Outer loop (on the GPU, FP64):   r = b - A x;  stop if |r| <= tol |r0|;
Inner solve (on the GPU, FP32):  e = `inner` Jacobi sweeps of A e = r from
                                 e = 0 (zero shell), t sweeps per pass;
Update (on the GPU, FP64):       x += e.
The only host synchronisation per outer iteration reads |r|^2 (8 bytes).
"""
import math

import numpy as np
import torch

from . import jacobi


def refine_solve(x, tol=1e-10, inner=50, t=8, max_outer=10**6, check_every=1, callback=None,
                 bx=0, by=0, waves=0, fused=True, state=None):
    """Solve in place.  x: float64 GPU grid (shell = Dirichlet data, interior
    = initial guess).  Returns (x, outer_iterations, relative_residual).
    ``check_every`` > 1 reads the norm only every that many outer iterations
    (fewer host synchronisations; the stopping point is then a multiple).
    t, bx, by, waves: blocking of the inner FP32 sweeps (t=None and 0: the
    library's choice).  ``fused``: update x and take the next residual in
    one pass over memory (x then alternates between two buffers, and the
    next inner solve's zero guess is written in the same pass); False runs
    the update, the residual and the zero fill as separate kernels.  Both
    give bitwise the same iterates.

    ``state``: a dict for checkpoint and resume.  On return it holds
    ``outer`` (outer iterations done, counted from the original start) and
    ``r0`` (the residual norm the tolerance is relative to).  Passed back in
    with those keys, beside the x that run returned, the solve continues
    where it stopped: the iterates, and so the final x and the outer count,
    are bitwise those of an uninterrupted run (max_outer counts from the
    original start too).  save_checkpoint / load_checkpoint keep both on
    disk."""
    if x.dtype != torch.float64:
        raise TypeError("x must be float64")
    r32 = torch.empty(x.shape, dtype=torch.float32, device=x.device)
    jacobi.fill(r32, 0.0)
    e_a = torch.empty_like(r32)
    e_b = torch.empty_like(r32)
    jacobi.fill(e_a, 0.0)
    jacobi.fill(e_b, 0.0)
    norm2 = torch.zeros(1, dtype=torch.float64, device=x.device)
    ws = jacobi.residual_workspace(x)
    xa, xb = x, (x.clone() if fused else None)
    jacobi.residual_f64(xa, r32, norm2, ws)
    r0 = None if state is None else state.get("r0")
    rel = float("inf")
    it = 0 if state is None else int(state.get("outer", 0))
    while True:
        if it % check_every == 0 or it >= max_outer:
            n = math.sqrt(norm2.item())
            if r0 is None:
                r0 = n if n > 0 else 1.0
            rel = n / r0
            if callback is not None:
                callback(it, rel)
            if rel <= tol or it >= max_outer:
                break
        # e_a holds zeros (interior and shell); e_b is scratch with a zero shell
        e = jacobi.tblock(e_a, e_b, inner, t=t, bx=bx, by=by, waves=waves, rhs=r32)
        other = e_b if e is e_a else e_a
        if fused:
            jacobi.update_residual_f64(xa, e, xb, r32, other, norm2, ws)
            xa, xb = xb, xa
        else:
            jacobi.update_f64(xa, e)
            jacobi.residual_f64(xa, r32, norm2, ws)
            jacobi.fill(other, 0.0)
        e_a, e_b = other, e
        it += 1
    if xa is not x:
        x.copy_(xa)
    if state is not None:
        state.update(outer=it, r0=r0)
    return x, it, rel


def save_checkpoint(path, x, state):
    """Write a stopped refinement (the grid x and its state dict) to an .npz
    file."""
    np.savez(path, x=x.detach().cpu().numpy(), outer=np.int64(state["outer"]),
             r0=np.float64(state["r0"]))


def load_checkpoint(path, device="cuda"):
    """(x on `device`, state) of a checkpoint written by save_checkpoint."""
    with np.load(path, allow_pickle=False) as f:
        x = torch.from_numpy(f["x"]).to(device)
        return x, {"outer": int(f["outer"]), "r0": float(f["r0"])}


def jacobi_solve_f64(x, tol=1e-10, check=50, t=None, max_sweeps=10**9, callback=None):
    """All-FP64 Jacobi (the update of Sect. 1.1) to |r| <= tol |r0|, the
    residual checked every ``check`` sweeps.  Returns (x, sweeps, rel).
    t: sweeps per blocked pass (None: the library's choice; 1: plain)."""
    if x.dtype != torch.float64:
        raise TypeError("x must be float64")
    a = x
    b = torch.empty_like(x)
    r32 = torch.empty(x.shape, dtype=torch.float32, device=x.device)
    norm2 = torch.zeros(1, dtype=torch.float64, device=x.device)
    ws = jacobi.residual_workspace(x)
    jacobi.residual_f64(a, r32, norm2, ws)
    r0 = math.sqrt(norm2.item()) or 1.0
    rel = 1.0
    sweeps = 0
    while rel > tol and sweeps < max_sweeps:
        out = jacobi.plain(a, b, check) if t == 1 else jacobi.tblock(a, b, check, t=t)
        if out is b:
            a, b = b, a
        sweeps += check
        jacobi.residual_f64(a, r32, norm2, ws)
        rel = math.sqrt(norm2.item()) / r0
        if callback is not None:
            callback(sweeps, rel)
    if a is not x:
        x.copy_(a)
    return x, sweeps, rel
