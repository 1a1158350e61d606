"""CPU oracle for the 3D Jacobi hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark import this package.  The product path neither imports it nor shares
code with it.  All arithmetic happens in the plain C library built from
``oracle.c`` (IEEE binary64, no FMA contraction); this module only marshals
numpy arrays.

Grids are C-contiguous float64 arrays of shape (nz+2, ny+2, nx+2): index
``u[k, j, i]``, i fastest, a one-cell Dirichlet shell on every face.

Functions and the passages they follow:
  sweeps       -- T Jacobi sweeps, update equation of Sect. 1.1, grids A and B
                  written in turn.
  point        -- level T at one cell from its domain of dependence (same
                  arithmetic as ``sweeps``; bitwise equal).
  rhs_sweeps   -- Jacobi sweeps for (6I - adjacency) e = r with a zero shell
                  (inner solve of the mixed-precision refinement).
  residual     -- r = b - A x of the Laplace system whose fixed point the
                  Jacobi iteration of Sect. 1.1 seeks.
  adjoint      -- gradient of a loss on level T with respect to level 0
                  (interior and shell) through the linear sweep operator.
  jacobi_solve -- all-FP64 Jacobi iteration to a relative residual tolerance.
  lbm_d3q19    -- time steps of the D3Q19 lattice Boltzmann method (BGK,
                  periodic box), the stencil method the paper takes the Jacobi
                  sweep as a prototype of (Sect. 1.1); with lbm_lattice and
                  lbm_equilibrium (lbm.c).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dbl_p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_L = ctypes.c_long


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build
        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_max_threads.argtypes = [ctypes.c_int]
    lib.oracle_max_threads.restype = ctypes.c_int
    lib.oracle_sweeps.argtypes = [_L, _L, _L, _dbl_p, _dbl_p, ctypes.c_int, ctypes.c_int]
    lib.oracle_sweeps.restype = ctypes.c_int
    lib.oracle_point.argtypes = [_L, _L, _L, _dbl_p, ctypes.c_int, _L, _L, _L]
    lib.oracle_point.restype = ctypes.c_double
    lib.oracle_rhs_sweeps.argtypes = [_L, _L, _L, _dbl_p, _dbl_p, ctypes.c_int, ctypes.c_int]
    lib.oracle_rhs_sweeps.restype = ctypes.c_int
    lib.oracle_residual.argtypes = [_L, _L, _L, _dbl_p, _dbl_p]
    lib.oracle_residual.restype = ctypes.c_double
    lib.oracle_adjoint.argtypes = [_L, _L, _L, _dbl_p, _dbl_p, ctypes.c_int, ctypes.c_int]
    lib.oracle_adjoint.restype = ctypes.c_int
    lib.oracle_jacobi_solve.argtypes = [_L, _L, _L, _dbl_p, ctypes.c_double, ctypes.c_int,
                                        _L, ctypes.c_int, ctypes.POINTER(_L),
                                        ctypes.POINTER(ctypes.c_double)]
    lib.oracle_jacobi_solve.restype = ctypes.c_int
    lib.oracle_copy_bandwidth.argtypes = [_L, ctypes.c_int, ctypes.c_int]
    lib.oracle_copy_bandwidth.restype = ctypes.c_double
    lib.oracle_lbm_lattice.argtypes = [np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS"),
                                       _dbl_p]
    lib.oracle_lbm_lattice.restype = None
    lib.oracle_lbm_equilibrium.argtypes = [ctypes.c_double] * 4 + [_dbl_p]
    lib.oracle_lbm_equilibrium.restype = None
    lib.oracle_lbm_d3q19.argtypes = [_L, _L, _L, _dbl_p, _dbl_p, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_int]
    lib.oracle_lbm_d3q19.restype = ctypes.c_int
    _lib = lib
    return lib


def _dims(u):
    if u.ndim != 3 or min(u.shape) < 3:
        raise ValueError(f"grid must be 3-D with every extent >= 3, got {u.shape}")
    nz, ny, nx = (s - 2 for s in u.shape)
    return nx, ny, nz


def _as_grid(u):
    return np.ascontiguousarray(u, dtype=np.float64)


def max_threads(nthreads=0):
    """OpenMP threads the oracle uses (nthreads <= 0: the runtime default)."""
    return _load().oracle_max_threads(nthreads)


def sweeps(u, T, nthreads=0):
    """Level T of the Jacobi iteration started from the full grid ``u``."""
    u = _as_grid(u)
    nx, ny, nz = _dims(u)
    out = np.empty_like(u)
    if _load().oracle_sweeps(nx, ny, nz, u, out, int(T), nthreads) != 0:
        raise ValueError("oracle_sweeps failed")
    return out


def point(u, T, i, j, k):
    """Level T at cell (i, j, k) (array indices, shell = 0 and n+1)."""
    u = _as_grid(u)
    nx, ny, nz = _dims(u)
    v = _load().oracle_point(nx, ny, nz, u, int(T), int(i), int(j), int(k))
    if np.isnan(v) and not np.isnan(u).any():
        raise ValueError("oracle_point: bad arguments")
    return v


def rhs_sweeps(r, T, nthreads=0):
    """T sweeps of e <- (sum of 6 neighbours + r) / 6 from e = 0, zero shell."""
    r = _as_grid(r)
    nx, ny, nz = _dims(r)
    out = np.empty_like(r)
    if _load().oracle_rhs_sweeps(nx, ny, nz, r, out, int(T), nthreads) != 0:
        raise ValueError("oracle_rhs_sweeps failed")
    return out


def residual(x):
    """(r, ||r||^2): r = sum of 6 neighbours - 6x on the interior, zero shell."""
    x = _as_grid(x)
    nx, ny, nz = _dims(x)
    r = np.empty_like(x)
    n2 = _load().oracle_residual(nx, ny, nz, x, r)
    return r, n2


def adjoint(grad_out, T, nthreads=0):
    """Gradient w.r.t. the level-0 grid (interior and shell) of a loss whose
    gradient w.r.t. level T is ``grad_out`` (full grid)."""
    g = _as_grid(grad_out)
    nx, ny, nz = _dims(g)
    out = np.empty_like(g)
    if _load().oracle_adjoint(nx, ny, nz, g, out, int(T), nthreads) != 0:
        raise ValueError("oracle_adjoint failed")
    return out


def jacobi_solve(x0, tol, check_every=50, max_sweeps=10**7, nthreads=0):
    """All-FP64 Jacobi from ``x0`` until ||r|| <= tol*||r0|| (checked every
    ``check_every`` sweeps).  Returns (x, sweeps, rel_res, converged)."""
    x = _as_grid(x0).copy()
    nx, ny, nz = _dims(x)
    done = _L(0)
    rel = ctypes.c_double(0.0)
    rc = _load().oracle_jacobi_solve(nx, ny, nz, x, float(tol), int(check_every),
                                     int(max_sweeps), nthreads, ctypes.byref(done),
                                     ctypes.byref(rel))
    if rc < 0:
        raise ValueError("oracle_jacobi_solve: bad arguments")
    return x, done.value, rel.value, rc == 0


def copy_bandwidth(n_doubles=1 << 27, reps=5, nthreads=0):
    """Host copy bandwidth in bytes/s (read + write), STREAM-COPY style: the
    M_s of the CPU baseline's Eq. 2 figure (not part of the method)."""
    bw = _load().oracle_copy_bandwidth(int(n_doubles), int(reps), nthreads)
    if bw < 0:
        raise MemoryError("oracle_copy_bandwidth: allocation failed")
    return bw


def lbm_lattice():
    """(c, w): the D3Q19 velocities (19 x 3 ints) and weights (19 doubles)."""
    c = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    _load().oracle_lbm_lattice(c, w)
    return c.reshape(19, 3), w


def lbm_equilibrium(rho, ux, uy, uz):
    """The 19 equilibrium populations of density rho and velocity (ux, uy, uz)."""
    out = np.zeros(19)
    _load().oracle_lbm_equilibrium(float(rho), float(ux), float(uy), float(uz), out)
    return out


def lbm_d3q19(f, omega, T, nthreads=0):
    """Populations after T lattice Boltzmann steps (stream, then BGK collision
    with rate omega) from ``f`` of shape (19, nz, ny, nx), periodic box."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    if f.ndim != 4 or f.shape[0] != 19:
        raise ValueError(f"populations must have shape (19, nz, ny, nx), got {f.shape}")
    _, nz, ny, nx = f.shape
    out = np.empty_like(f)
    if _load().oracle_lbm_d3q19(nx, ny, nz, f, out, float(omega), int(T), nthreads) != 0:
        raise ValueError("oracle_lbm_d3q19 failed")
    return out
