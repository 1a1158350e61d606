"""Pins of the oracle's adjoint, residual, right-hand-side sweeps and Jacobi
solve against the mathematics: dense matrices built from the grid graph, the
dot-product (transpose) identity, finite differences, discrete harmonic
polynomials and a spectral (DST-I) direct solve."""
import math

import numpy as np
import pytest
import scipy.fft

from paper_0912_4506_amd import inputs
from test_oracle_pins import bound, dense_operator, interior_cells, to_vec, harmonic, U


def full_sweep_matrix(nx, ny, nz):
    """One sweep as a (full -> full) matrix: interior rows (Adj|Bnd)/6, shell rows identity."""
    cells, adj, bnd = dense_operator(nx, ny, nz)
    nfull = (nx + 2) * (ny + 2) * (nz + 2)
    S = np.eye(nfull)
    for r, (i, j, k) in enumerate(cells):
        p = i + (nx + 2) * (j + (ny + 2) * k)
        S[p, :] = bnd[r] / 6.0
        for c, (i2, j2, k2) in enumerate(cells):
            if adj[r, c]:
                S[p, i2 + (nx + 2) * (j2 + (ny + 2) * k2)] += adj[r, c] / 6.0
    return S


@pytest.mark.parametrize("shape,T", [((2, 3, 2), 1), ((3, 2, 4), 4), ((1, 2, 3), 3)])
def test_adjoint_dense_transpose(oracle_mod, shape, T):
    nx, ny, nz = shape
    S = full_sweep_matrix(nx, ny, nz)
    J = np.linalg.matrix_power(S, T)
    lam = np.random.default_rng(1).random(((nz + 2), (ny + 2), (nx + 2)))
    got = oracle_mod.adjoint(lam, T)
    ref = (J.T @ lam.ravel()).reshape(lam.shape)
    assert np.max(np.abs(got - ref)) <= 4 * bound(T, 1.0) * T + 8 * U
    # the forward oracle agrees with the same matrix (sanity of the matrix)
    u = inputs.grid(nx, ny, nz, seed=2)
    assert np.max(np.abs(oracle_mod.sweeps(u, T).ravel() - J @ u.ravel())) <= 2 * bound(T, 1.0)


def test_adjoint_dot_product_identity(oracle_mod):
    """<F_T(d), lam> = <d, F_T^*(lam)> with F_T the (linear) forward oracle."""
    nx, ny, nz, T = 12, 9, 10, 11
    rng = np.random.default_rng(7)
    d = rng.random((nz + 2, ny + 2, nx + 2)) - 0.5
    lam = rng.random(d.shape) - 0.5
    lhs = np.sum(oracle_mod.sweeps(d, T) * lam)
    rhs = np.sum(d * oracle_mod.adjoint(lam, T))
    assert abs(lhs - rhs) <= 1e-12 * np.sum(np.abs(d)) * np.max(np.abs(lam))


def test_adjoint_finite_differences_quadratic(oracle_mod):
    """L = sum w * A_T^2 is quadratic, so the central difference is exact up to
    roundoff for any step h; shell edges and corners get exactly zero."""
    nx, ny, nz, T = 6, 5, 7, 6
    u = inputs.grid(nx, ny, nz, seed=0)
    w = inputs.adjoint_weights(nx, ny, nz, seed=0)

    def loss(v):
        a = oracle_mod.sweeps(v, T)
        return float(np.sum(w * a * a))

    g = oracle_mod.adjoint(2 * w * oracle_mod.sweeps(u, T), T)
    rng = np.random.default_rng(3)
    cells = [(int(rng.integers(1, nx + 1)), int(rng.integers(1, ny + 1)), int(rng.integers(1, nz + 1)))
             for _ in range(6)]
    cells += [(0, 2, 3), (nx + 1, 1, 1), (3, 0, 2), (2, ny + 1, 5), (4, 4, 0), (1, 3, nz + 1)]
    cells += [(0, 0, 3), (nx + 1, ny + 1, nz + 1), (0, 2, 0)]          # edges / corner
    h = 1e-2
    gmax = np.max(np.abs(g))
    for (i, j, k) in cells:
        up, dn = u.copy(), u.copy()
        up[k, j, i] += h
        dn[k, j, i] -= h
        fd = (loss(up) - loss(dn)) / (2 * h)
        assert abs(fd - g[k, j, i]) <= 1e-9 * gmax, (i, j, k, fd, g[k, j, i])
    for (i, j, k) in [(0, 0, 3), (nx + 1, ny + 1, nz + 1), (0, 2, 0)]:
        assert g[k, j, i] == 0.0


def test_adjoint_interior_is_zero_shell_forward(oracle_mod):
    """M is symmetric, so the interior adjoint equals the forward sweeps of the
    interior gradient with a zero shell (bitwise: same operations)."""
    nx, ny, nz, T = 9, 8, 10, 7
    lam = np.random.default_rng(4).random((nz + 2, ny + 2, nx + 2))
    z = np.zeros_like(lam)
    z[1:-1, 1:-1, 1:-1] = lam[1:-1, 1:-1, 1:-1]
    a = oracle_mod.adjoint(lam, T)
    f = oracle_mod.sweeps(z, T)
    assert np.array_equal(a[1:-1, 1:-1, 1:-1], f[1:-1, 1:-1, 1:-1])
    # T = 0: identity
    assert np.array_equal(oracle_mod.adjoint(lam, 0), lam)


def test_residual_pins(oracle_mod):
    nx, ny, nz = 7, 6, 8
    k, j, i = np.meshgrid(np.arange(nz + 2), np.arange(ny + 2), np.arange(nx + 2), indexing="ij")
    p = harmonic(i, j, k).astype(np.float64)
    r, n2 = oracle_mod.residual(p)
    assert np.all(r == 0) and n2 == 0.0
    # zero interior: r = b = sum of the shell neighbours (sign and scale of b - A x)
    g = inputs.laplace_problem(nx, ny, nz, seed=5)
    cells, adj, bnd = dense_operator(nx, ny, nz)
    r, n2 = oracle_mod.residual(g)
    b = bnd @ g.ravel()
    assert np.max(np.abs(to_vec(r, cells) - b)) <= 8 * U * 6
    # general x: r = b + Adj x - 6 x
    x = inputs.grid(nx, ny, nz, seed=6)
    r, n2 = oracle_mod.residual(x)
    ref = bnd @ x.ravel() + adj @ to_vec(x, cells) - 6 * to_vec(x, cells)
    assert np.max(np.abs(to_vec(r, cells) - ref)) <= 16 * U * 12
    assert math.isclose(n2, float(np.sum(ref ** 2)), rel_tol=1e-12)
    mask = np.ones(r.shape, bool)
    mask[1:-1, 1:-1, 1:-1] = False
    assert np.all(r[mask] == 0)


def dst_solve(b_int):
    """Direct solve of (6I - adjacency) x = b on the interior with zero
    Dirichlet data: orthonormal DST-I diagonalises the operator."""
    nz, ny, nx = b_int.shape
    ck = np.cos(np.pi * np.arange(1, nz + 1) / (nz + 1))
    cj = np.cos(np.pi * np.arange(1, ny + 1) / (ny + 1))
    ci = np.cos(np.pi * np.arange(1, nx + 1) / (nx + 1))
    eig = 6 - 2 * (ck[:, None, None] + cj[None, :, None] + ci[None, None, :])
    bh = scipy.fft.dstn(b_int, type=1, norm="ortho")
    return scipy.fft.dstn(bh / eig, type=1, norm="ortho")


def test_rhs_sweeps_pins(oracle_mod):
    nx, ny, nz, T = 4, 3, 5, 6
    r = inputs.grid(nx, ny, nz, seed=9)
    cells, adj, bnd = dense_operator(nx, ny, nz)
    e = np.zeros(len(cells))
    rv = to_vec(r, cells)
    for _ in range(T):
        e = (adj @ e + rv) / 6.0
    got = oracle_mod.rhs_sweeps(r, T)
    assert np.max(np.abs(to_vec(got, cells) - e)) <= 2 * bound(T, 2 * T)
    mask = np.ones(r.shape, bool)
    mask[1:-1, 1:-1, 1:-1] = False
    assert np.all(got[mask] == 0)
    # many sweeps converge to the direct solution of (6I - Adj) e = r
    nx, ny, nz = 6, 5, 7
    r = inputs.grid(nx, ny, nz, seed=10)
    got = oracle_mod.rhs_sweeps(r, 2000)
    x = dst_solve(r[1:-1, 1:-1, 1:-1])
    assert np.max(np.abs(got[1:-1, 1:-1, 1:-1] - x)) <= 1e-10 * np.max(np.abs(x))


def test_jacobi_solve_vs_dst(oracle_mod):
    nx, ny, nz = 10, 9, 12
    g = inputs.laplace_problem(nx, ny, nz, seed=0)
    cells, adj, bnd = dense_operator(nx, ny, nz)
    b = (bnd @ g.ravel())
    b_int = np.zeros((nz, ny, nx))
    for n, (i, j, k) in enumerate(cells):
        b_int[k - 1, j - 1, i - 1] = b[n]
    x_ref = dst_solve(b_int)
    x, sweeps, rel, ok = oracle_mod.jacobi_solve(g, 1e-10, check_every=50)
    assert ok and rel <= 1e-10 and sweeps % 50 == 0
    lam_min = 6 - 2 * (math.cos(math.pi / (nx + 1)) + math.cos(math.pi / (ny + 1))
                       + math.cos(math.pi / (nz + 1)))
    err_bound = rel * np.linalg.norm(b) / lam_min
    assert np.max(np.abs(x[1:-1, 1:-1, 1:-1] - x_ref)) <= 1.01 * err_bound
    # shell unchanged
    mask = np.ones(g.shape, bool)
    mask[1:-1, 1:-1, 1:-1] = False
    assert np.array_equal(x[mask], g[mask])
    # the sweep count follows the slowest mode: rho = (sum of cos(pi/(n+1)))/3
    rho = (math.cos(math.pi / (nx + 1)) + math.cos(math.pi / (ny + 1))
           + math.cos(math.pi / (nz + 1))) / 3
    predicted = math.log(1e-10) / math.log(rho)
    assert 0.5 * predicted <= sweeps <= 1.5 * predicted + 50


def test_jacobi_solve_harmonic_shell(oracle_mod):
    """A discrete harmonic polynomial on the shell: the solution is the
    polynomial itself."""
    nx, ny, nz = 8, 7, 9
    k, j, i = np.meshgrid(np.arange(nz + 2), np.arange(ny + 2), np.arange(nx + 2), indexing="ij")
    p = (i * j - 2 * j * k + 3 * i - k + i * j * k / 10.0).astype(np.float64)
    x0 = p.copy()
    x0[1:-1, 1:-1, 1:-1] = 0.0
    x, sweeps, rel, ok = oracle_mod.jacobi_solve(x0, 1e-11, check_every=50)
    assert ok
    assert np.max(np.abs(x - p)) <= 1e-8 * np.max(np.abs(p))
