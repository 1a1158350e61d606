"""Seeded synthetic inputs for the Jacobi workloads.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic.  Tests hand the same arrays to the GPU path and to the CPU
oracle; the benchmark draws its inputs here too.

Recipe (the paper measures a 600^3 double-precision grid and publishes no data
set; every workload here is synthetic):
  * grid(nx, ny, nz, seed): ``default_rng(seed).random((nz+2, ny+2, nx+2))``,
    float64 uniform on [0, 1), one draw covering interior and shell; i is the
    fastest axis.  A float32 grid is the float64 draw rounded with ``astype``.
  * laplace_problem: the same draw with the interior set to zero (Dirichlet
    data uniform on [0, 1), zero initial guess).
  * adjoint_weights: ``default_rng(seed + 1)`` uniform [0, 1) over the
    interior, zero on the shell.
  * batch_edges: 64 cubic interior edges, e = clip(round(exp(U(ln 32, ln 256))),
    32, 256) from ``default_rng(seed)``; ``cubic=False`` draws the three axes
    independently.  Grid g of a batch is ``grid(..., seed=[seed, g])``.
  * lbm_populations(nx, ny, nz, seed): 19 arrays of (nz, ny, nx) values
    (1 + 0.1 U[0, 1)) / 19 from ``default_rng(seed)``: positive populations
    with density near 1 and a small random velocity, far from equilibrium
    (the lattice Boltzmann workload; its time per step does not depend on the
    values).
"""
import math

import numpy as np


def grid(nx, ny, nz, seed=0, dtype=np.float64):
    """Full (nz+2, ny+2, nx+2) grid, uniform [0, 1) interior and shell."""
    rng = np.random.default_rng(seed)
    u = rng.random((nz + 2, ny + 2, nx + 2))
    return u.astype(dtype, copy=False)


def laplace_problem(nx, ny, nz, seed=0, dtype=np.float64):
    """Grid whose shell is uniform [0, 1) Dirichlet data and interior is 0."""
    u = grid(nx, ny, nz, seed, np.float64)
    u[1:-1, 1:-1, 1:-1] = 0.0
    return u.astype(dtype, copy=False)


def adjoint_weights(nx, ny, nz, seed=0, dtype=np.float64):
    """Loss weights w: uniform [0, 1) on the interior, 0 on the shell."""
    rng = np.random.default_rng(seed + 1)
    w = np.zeros((nz + 2, ny + 2, nx + 2))
    w[1:-1, 1:-1, 1:-1] = rng.random((nz, ny, nx))
    return w.astype(dtype, copy=False)


def batch_edges(n=64, seed=0, lo=32, hi=256, cubic=True):
    """List of (nx, ny, nz) interior extents, log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)

    def draw(size):
        e = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size)))
        return np.clip(e, lo, hi).astype(int)

    if cubic:
        return [(int(e), int(e), int(e)) for e in draw(n)]
    return [tuple(int(v) for v in row) for row in draw((n, 3))]


def batch_grid(shape, index, seed=0, dtype=np.float64):
    """Grid ``index`` of a batch: uniform [0, 1) from ``default_rng([seed, index])``."""
    nx, ny, nz = shape
    return grid(nx, ny, nz, seed=[seed, index], dtype=dtype)


def lbm_populations(nx, ny, nz, seed=0, dtype=np.float64):
    """(19, nz, ny, nx) positive populations, (1 + 0.1 U[0, 1)) / 19."""
    rng = np.random.default_rng(seed)
    f = (1.0 + 0.1 * rng.random((19, nz, ny, nx))) / 19.0
    return f.astype(dtype, copy=False)
