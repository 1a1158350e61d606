"""Pins of the CPU oracle's forward sweep against facts fixed by the
mathematics of the Jacobi update (update equation of Sect. 1.1), never against
the oracle's own formula.

Each test is chosen so that a plausible slip in the oracle (a dropped or
doubled neighbour, a shifted index, a wrong sign, a transposed axis, a wrong
divisor, a wrong buffer swap) fails at least one of them.

Error bound used throughout: one sweep adds at most 5 roundings of partial
sums bounded by 6*max|u| plus one rounding of the division, i.e.
(2+3+4+5+6)/6*u + u < 4.4u relative to max|u| (u = 2^-53), and the sweep is
non-expansive, so T sweeps stay within 4.4*T*u*max|u| of the exact result.
"""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_0912_4506_amd import inputs

U = 2.0 ** -53


def bound(T, scale):
    return 4.4 * T * U * scale


# ---------------------------------------------------------------- helpers ---
def interior_cells(nx, ny, nz):
    return [(i, j, k) for k in range(1, nz + 1) for j in range(1, ny + 1)
            for i in range(1, nx + 1)]


NEIGH = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]


def dense_operator(nx, ny, nz):
    """Interior adjacency (integer) and interior-to-shell coupling built from
    the grid graph: (Adj x + Bnd g) / 6 is one sweep."""
    cells = interior_cells(nx, ny, nz)
    pos = {c: n for n, c in enumerate(cells)}
    full = [(i, j, k) for k in range(nz + 2) for j in range(ny + 2) for i in range(nx + 2)]
    fpos = {c: n for n, c in enumerate(full)}
    adj = np.zeros((len(cells), len(cells)))
    bnd = np.zeros((len(cells), len(full)))
    for c in cells:
        for d in NEIGH:
            q = (c[0] + d[0], c[1] + d[1], c[2] + d[2])
            if q in pos:
                adj[pos[c], pos[q]] += 1
            else:
                bnd[pos[c], fpos[q]] += 1
    return cells, adj, bnd


def to_vec(u, cells):
    return np.array([u[k, j, i] for (i, j, k) in cells])


# ----------------------------------------------------------------- tests ---
def test_single_cell_closed_form(oracle_mod):
    """A 1x1x1 interior: one sweep is the mean of the six face values."""
    u = np.zeros((3, 3, 3))
    u[1, 1, 0], u[1, 1, 2] = 1.0, 2.0          # i-1, i+1
    u[1, 0, 1], u[1, 2, 1] = 3.0, 4.0          # j-1, j+1
    u[0, 1, 1], u[2, 1, 1] = 5.0, 6.0          # k-1, k+1
    u[1, 1, 1] = 1000.0                        # no centre term
    out = oracle_mod.sweeps(u, 1)
    assert out[1, 1, 1] == 3.5
    # the shell is untouched, and a second sweep gives the same value
    centre = np.zeros(u.shape, bool)
    centre[1, 1, 1] = True
    assert np.array_equal(out[~centre], u[~centre])
    assert oracle_mod.sweeps(u, 2)[1, 1, 1] == 3.5
    # a non-integer mean is the correctly rounded quotient
    u[1, 1, 0] = 2.0
    assert oracle_mod.sweeps(u, 1)[1, 1, 1] == 22.0 / 6.0
    # T = 0 is the identity
    assert np.array_equal(oracle_mod.sweeps(u, 0), u)


def test_division_is_correctly_rounded(oracle_mod):
    """The divide by 6 is one correctly rounded IEEE division: for sums where
    multiplying by the rounded reciprocal 1/6 lands on the neighbouring double,
    the oracle must give the exactly rounded rational s/6."""
    for s in (871.0390625, 652.2490234375, 41.95703125, 179.4736328125, 665.001953125):
        assert s * (1.0 / 6.0) != float(Fraction(s) / 6)   # the case is discriminating
        u = np.zeros((3, 3, 3))
        u[1, 1, 0] = s                                      # the exact sum of the six faces
        assert oracle_mod.sweeps(u, 1)[1, 1, 1] == float(Fraction(s) / 6)


@pytest.mark.parametrize("shape,T", [((3, 2, 2), 1), ((2, 3, 4), 3), ((4, 3, 2), 6),
                                      ((1, 5, 2), 4)])
def test_dense_matrix(oracle_mod, shape, T):
    """x_{s} = (Adj x_{s-1} + Bnd g) / 6 with the matrices built from the grid graph."""
    nx, ny, nz = shape
    u = inputs.grid(nx, ny, nz, seed=11)
    cells, adj, bnd = dense_operator(nx, ny, nz)
    x = to_vec(u, cells)
    g = u.ravel()
    for _ in range(T):
        x = (adj @ x + bnd @ g) / 6.0
    out = oracle_mod.sweeps(u, T)
    got = to_vec(out, cells)
    assert np.max(np.abs(got - x)) <= 2 * bound(T, 1.0)
    # the shell is carried over unchanged
    mask = np.ones(u.shape, bool)
    mask[1:-1, 1:-1, 1:-1] = False
    assert np.array_equal(out[mask], u[mask])


def test_exact_rationals(oracle_mod):
    """Brute force in exact rational arithmetic on a tiny grid."""
    nx, ny, nz, T = 3, 2, 4, 5
    rng = np.random.default_rng(5)
    ints = rng.integers(0, 1024, size=(nz + 2, ny + 2, nx + 2))
    u = ints / 1024.0
    exact = {(i, j, k): Fraction(int(ints[k, j, i]), 1024)
             for k in range(nz + 2) for j in range(ny + 2) for i in range(nx + 2)}
    for _ in range(T):
        nxt = dict(exact)
        for c in interior_cells(nx, ny, nz):
            nxt[c] = sum(exact[(c[0] + d[0], c[1] + d[1], c[2] + d[2])] for d in NEIGH) / 6
        exact = nxt
    out = oracle_mod.sweeps(u, T)
    err = max(abs(Fraction(float(out[k, j, i])) - exact[(i, j, k)])
              for (i, j, k) in interior_cells(nx, ny, nz))
    assert float(err) <= bound(T, 1.0)
    # and the exact first sweep is reproduced to within one rounding chain
    out1 = oracle_mod.sweeps(u, 1)
    assert np.isclose(out1[2, 1, 2], float(sum(Fraction(int(ints[2 + d[2], 1 + d[1], 2 + d[0]]), 1024)
                                                 for d in NEIGH) / 6), rtol=0, atol=bound(1, 1))


@pytest.mark.parametrize("n,mode,T", [((20, 20, 20), (1, 1, 1), 50),
                                      ((20, 20, 20), (20, 20, 20), 51),
                                      ((24, 17, 30), (1, 2, 3), 100),
                                      ((13, 9, 7), (4, 9, 2), 40),
                                      ((63, 63, 63), (32, 32, 32), 5)])
def test_eigenmodes(oracle_mod, n, mode, T):
    """sin-mode eigenvectors with a zero shell: level T = lambda^T * v with
    lambda = (cos(pi a/(nx+1)) + cos(pi b/(ny+1)) + cos(pi c/(nz+1))) / 3."""
    nx, ny, nz = n
    a, b, c = mode
    i = np.arange(nx + 2)
    j = np.arange(ny + 2)
    k = np.arange(nz + 2)
    v = (np.sin(np.pi * c * k / (nz + 1))[:, None, None]
         * np.sin(np.pi * b * j / (ny + 1))[None, :, None]
         * np.sin(np.pi * a * i / (nx + 1))[None, None, :])
    v[0], v[-1], v[:, 0], v[:, -1], v[:, :, 0], v[:, :, -1] = 0, 0, 0, 0, 0, 0
    lam = (math.cos(math.pi * a / (nx + 1)) + math.cos(math.pi * b / (ny + 1))
           + math.cos(math.pi * c / (nz + 1))) / 3
    out = oracle_mod.sweeps(v, T)
    # error measured against max|v|: when |lambda|^T << u, roundoff in v excites
    # slower modes, so a bound relative to lambda^T would be meaningless
    err = np.max(np.abs(out - lam ** T * v))
    assert err <= bound(T, 1.0) + 16 * U
    # the wrong eigenvalue (say a sum over 6 terms with one axis doubled) is far off
    assert abs(lam) < 1


def harmonic(i, j, k):
    return 3 * i * j - 2 * j * k + i * i - k * k + 5 * i * j * k + 7


def test_harmonic_polynomial_fixed_point_bitwise(oracle_mod):
    """Discrete harmonic polynomials are exact fixed points: the six
    neighbours sum to 6p exactly in integers, and 6p/6 = p exactly."""
    nx, ny, nz = 30, 20, 25
    k, j, i = np.meshgrid(np.arange(nz + 2), np.arange(ny + 2), np.arange(nx + 2), indexing="ij")
    p = harmonic(i, j, k).astype(np.float64)
    assert np.array_equal(oracle_mod.sweeps(p, 20), p)
    # each pure monomial pins one neighbour pair: i^2 - k^2 pins i+-1 and k+-1,
    # ijk pins all three axes, ij - j^2 + ... etc.
    for q in (i * i - j * j, j * j - k * k, i * j * k, i - 2 * j + 3 * k):
        q = q.astype(np.float64)
        assert np.array_equal(oracle_mod.sweeps(q, 3), q)
    # a non-harmonic field (i^2) is NOT fixed: guards against a vacuous test
    q = (i * i).astype(np.float64)
    assert not np.array_equal(oracle_mod.sweeps(q, 1), q)
    # constants with a short mantissa are fixed
    c = np.full((nz + 2, ny + 2, nx + 2), 0.8125)
    assert np.array_equal(oracle_mod.sweeps(c, 7), c)


@pytest.mark.parametrize("T", [1, 4, 7])
def test_nan_cone(oracle_mod, T):
    """One interior NaN reaches exactly the interior cells at L1 distance
    d <= T with d = T (mod 2): the update has no centre term."""
    nx, ny, nz = 11, 9, 10
    u = inputs.grid(nx, ny, nz, seed=3)
    p = (5, 4, 6)
    u[p[2], p[1], p[0]] = np.nan
    out = oracle_mod.sweeps(u, T)
    k, j, i = np.meshgrid(np.arange(nz + 2), np.arange(ny + 2), np.arange(nx + 2), indexing="ij")
    d = np.abs(i - p[0]) + np.abs(j - p[1]) + np.abs(k - p[2])
    inner = (i >= 1) & (i <= nx) & (j >= 1) & (j <= ny) & (k >= 1) & (k <= nz)
    expect = inner & (d <= T) & (d % 2 == T % 2)
    assert np.array_equal(np.isnan(out), expect)


def test_monotone_and_max_principle(oracle_mod):
    """u <= v pointwise implies sweep(u) <= sweep(v) bitwise (round to nearest
    is monotone); values stay within [min, max] of the data."""
    nx, ny, nz, T = 14, 10, 12, 9
    u = inputs.grid(nx, ny, nz, seed=21)
    v = u + np.random.default_rng(22).random(u.shape) * 1e-3
    a = oracle_mod.sweeps(u, T)
    b = oracle_mod.sweeps(v, T)
    assert np.all(a <= b)
    assert a.min() >= u.min() and a.max() <= u.max()


def test_i_reflection_bitwise(oracle_mod):
    """Mirroring the grid in i mirrors the result bitwise: only the first
    addition sees the two i-neighbours, and it commutes."""
    nx, ny, nz, T = 9, 7, 8, 6
    u = inputs.grid(nx, ny, nz, seed=8)
    a = oracle_mod.sweeps(u, T)
    b = oracle_mod.sweeps(u[:, :, ::-1].copy(), T)
    assert np.array_equal(a[:, :, ::-1], b)


def test_axis_permutation(oracle_mod):
    """Swapping axes permutes the result (up to summation order)."""
    nx, ny, nz, T = 6, 8, 5, 7
    u = inputs.grid(nx, ny, nz, seed=9)
    a = oracle_mod.sweeps(u, T)
    for perm in itertools.permutations(range(3)):
        b = oracle_mod.sweeps(np.ascontiguousarray(u.transpose(perm)), T)
        assert np.max(np.abs(b - a.transpose(perm))) <= 2 * bound(T, 1.0)


def test_linearity(oracle_mod):
    """A_T(u, g) = A_T(u, 0) + A_T(0, g) and A_T(2u) = 2 A_T(u) (the latter bitwise)."""
    nx, ny, nz, T = 10, 12, 9, 8
    u = inputs.grid(nx, ny, nz, seed=4)
    inner = np.zeros_like(u)
    inner[1:-1, 1:-1, 1:-1] = u[1:-1, 1:-1, 1:-1]
    shell = u - inner
    a = oracle_mod.sweeps(u, T)
    b = oracle_mod.sweeps(inner, T) + oracle_mod.sweeps(shell, T)
    assert np.max(np.abs(a - b)) <= 3 * bound(T, 1.0)
    assert np.array_equal(oracle_mod.sweeps(2 * u, T), 2 * a)


def test_edges_and_corners_unread(oracle_mod):
    """Shell edges and corners have no interior neighbour: changing them
    changes nothing but themselves."""
    nx, ny, nz, T = 5, 6, 7, 5
    u = inputs.grid(nx, ny, nz, seed=2)
    v = u.copy()
    k, j, i = np.meshgrid(np.arange(nz + 2), np.arange(ny + 2), np.arange(nx + 2), indexing="ij")
    on = (i == 0) | (i == nx + 1), (j == 0) | (j == ny + 1), (k == 0) | (k == nz + 1)
    edge = (on[0].astype(int) + on[1] + on[2]) >= 2
    v[edge] = 123.0
    a = oracle_mod.sweeps(u, T)
    b = oracle_mod.sweeps(v, T)
    assert np.array_equal(a[~edge], b[~edge])


def test_point_matches_sweeps_bitwise(oracle_mod):
    """The single-cell routine reproduces the full sweeps bitwise, including
    cells whose domain of dependence is clipped by the shell."""
    nx, ny, nz, T = 13, 11, 12, 7
    u = inputs.grid(nx, ny, nz, seed=6)
    full = oracle_mod.sweeps(u, T)
    rng = np.random.default_rng(0)
    pts = [(1, 1, 1), (nx, ny, nz), (1, ny, 6), (7, 6, 6), (0, 3, 3)]
    pts += [tuple(int(rng.integers(1, n + 1)) for n in (nx, ny, nz)) for _ in range(10)]
    for (i, j, k) in pts:
        assert oracle_mod.point(u, T, i, j, k) == full[k, j, i]
    assert oracle_mod.point(u, 0, 4, 4, 4) == u[4, 4, 4]


def test_thread_count_does_not_change_bits(oracle_mod):
    nx, ny, nz, T = 17, 15, 16, 5
    u = inputs.grid(nx, ny, nz, seed=12)
    a = oracle_mod.sweeps(u, T, nthreads=1)
    b = oracle_mod.sweeps(u, T, nthreads=4)
    assert np.array_equal(a, b)
