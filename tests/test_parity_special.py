"""GPU parity on special and extreme FP64 values, against the CPU oracle
(IEEE arithmetic in the printed order), through the C ABI.

The library's arithmetic contract (include/jacobi.h, "Arithmetic"):
  * jacobi_plain and the adjoint's shell-face gradient divide as IEEE division
    does for every input: bitwise, NaN where the oracle has NaN, the same
    infinities, signed zeros kept;
  * the blocked passes (tblock, RHS, adjoint interior, batched) are bitwise
    wherever the sums are finite and the quotients zero or normal; an infinite
    sum gives NaN instead of the infinity, and quotients in the subnormal range
    may be one step (2^-1074) off, a difference later levels carry along.
The cases: infinities and NaN in the interior and in the shell, a grid of
negative zeros, data scaled by 2^1000 (large, finite sums), by 2^1022 (sums
that overflow) and by 2^-1060 (every value subnormal).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0912_4506_amd import inputs

pytestmark = pytest.mark.gpu

SHAPE = (70, 45, 33)     # two 64-lane blocks along i at every depth, ragged j and k tails
T = 10
TINY = 2.0 ** -1074


def dev(u):
    return torch.from_numpy(np.ascontiguousarray(u)).to("cuda")


def case(name, seed=0):
    nx, ny, nz = SHAPE
    u = inputs.grid(nx, ny, nz, seed=seed)
    if name == "inf_interior":
        u[10, 20, 30] = np.inf
        u[25, 7, 64] = -np.inf
        u[5, 40, 3] = np.nan
    elif name == "inf_shell":
        u[0, 20, 30] = np.inf          # k = 0 face
        u[17, 0, 50] = -np.inf         # j = 0 face
        u[9, 30, nx + 1] = np.inf      # i = nx+1 face
        u[nz + 1, ny + 1, 0] = np.nan  # a corner: never read
    elif name == "neg_zero":
        u[:] = -0.0
        u[:, :, : nx // 3] = 0.0       # a +0 slab: sums of +0 and -0 are +0
    elif name == "huge":
        u *= 2.0 ** 1000
    elif name == "overflow":
        u *= 2.0 ** 1022               # sums of six values reach 2^1024: infinite
    elif name == "subnormal":
        u *= 2.0 ** -1060              # every value subnormal
    else:
        raise ValueError(name)
    return u


CASES = ["inf_interior", "inf_shell", "neg_zero", "huge", "overflow", "subnormal"]


def bits(x):
    return np.ascontiguousarray(x).view(np.uint64)


def check_exact(got, ref):
    """IEEE everywhere: NaN where the oracle has NaN, every other value
    bitwise (infinities and signed zeros included)."""
    nan = np.isnan(ref)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(bits(got[~nan]), bits(ref[~nan]))


def check_blocked(got, ref, steps):
    """The blocked passes' contract: the same finite cells; where the oracle
    is infinite, NaN or the same infinity; NaN where it is NaN; finite cells
    bitwise, or within 2 subnormal steps per level where the data reach the
    subnormal range."""
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin)
    inf = np.isinf(ref)
    assert np.all(np.isnan(got[inf]) | (got[inf] == ref[inf]))
    assert np.all(np.isnan(got[np.isnan(ref)]))
    if np.any(np.abs(ref[fin]) < 2.0 ** -1021):
        assert np.max(np.abs(got[fin] - ref[fin])) <= 2 * steps * TINY
    else:
        assert np.array_equal(bits(got[fin]), bits(ref[fin]))


@pytest.mark.parametrize("name", CASES)
def test_plain_is_ieee(jac, name):
    u = case(name)
    ref = oracle.sweeps(u, T)
    a = dev(u)
    b = torch.full_like(a, 7.0)
    out = jac.plain(a, b, T)
    torch.cuda.synchronize()
    check_exact(out.cpu().numpy(), ref)


@pytest.mark.parametrize("name", CASES)
def test_blocked_every_depth(jac, name):
    u = case(name)
    ref = oracle.sweeps(u, T)
    for t in range(1, 9):
        a = dev(u)
        out = jac.tblock(a, torch.full_like(a, 7.0), T, t=t)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        check_blocked(got, ref, T)
        if name in ("huge", "neg_zero"):     # finite sums, normal or zero quotients
            check_exact(got, ref)


@pytest.mark.parametrize("name", ["inf_interior", "huge", "subnormal", "neg_zero"])
def test_rhs_sweeps(jac, name):
    """Sweeps with a right-hand side (zero guess, zero shell) on special r."""
    r = case(name)
    ref = oracle.rhs_sweeps(r, T)
    a = torch.zeros(r.shape, dtype=torch.float64, device="cuda")
    for t in (1, 3, 5):
        out = jac.tblock(a.clone(), torch.full_like(a, 7.0), T, t=t, rhs=dev(r))
        torch.cuda.synchronize()
        check_blocked(out.cpu().numpy(), ref, T)


@pytest.mark.parametrize("name", ["inf_interior", "inf_shell", "huge", "overflow", "subnormal"])
def test_adjoint(jac, name):
    """The adjoint of T sweeps on a special gradient: interior by the blocked
    passes, shell faces by the IEEE-exact face kernel."""
    lam = case(name, seed=4)
    ref = oracle.adjoint(lam, T)
    a = dev(lam)
    out = jac.adjoint(a, torch.full_like(a, 7.0), T, t=4)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    check_blocked(got, ref, T + 1)
    # the shell faces come from G + S/6 with an IEEE division: where S is
    # finite they are bitwise (given bitwise traced levels)
    nz, ny, nx = (s - 2 for s in lam.shape)
    face = np.zeros(lam.shape, bool)
    face[0, 1:-1, 1:-1] = face[-1, 1:-1, 1:-1] = True
    face[1:-1, 0, 1:-1] = face[1:-1, -1, 1:-1] = True
    face[1:-1, 1:-1, 0] = face[1:-1, 1:-1, -1] = True
    if name == "huge":
        check_exact(got[face], ref[face])


def test_batched(jac):
    """A batch holding every special case (relaxed persistent launch)."""
    us = [case(n, seed=m) for m, n in enumerate(CASES)]
    a = [dev(u) for u in us]
    b = [torch.full_like(x, 7.0) for x in a]
    plan = jac.BatchPlan(a, b, [T] * len(us), t=5, bx=64, by=48)
    plan.run("relaxed")
    torch.cuda.synchronize()
    assert not plan.wait_error()
    for name, u, out in zip(CASES, us, plan.results()):
        ref = oracle.sweeps(u, T)
        got = out.cpu().numpy()
        check_blocked(got, ref, T)
        if name in ("huge", "neg_zero"):
            check_exact(got, ref)


def test_division_column(jac):
    """One sweep of a 1 x 1 x N column whose i-1 shell face carries the whole
    sum s (the other five neighbours are +0): the plain kernel's quotient is
    IEEE s/6 for every s; the blocked kernel's equals it wherever s/6 is zero
    or normal, is NaN for s = +-Inf, and within one step in the subnormal
    range."""
    rng = np.random.default_rng(0)
    s = np.concatenate([
        rng.random(1024) * 6.0,
        rng.integers(1, 2 ** 20, 512) / 1024.0,
        np.ldexp(1.0 + rng.random(512), rng.integers(-1022, 1020, 512)),     # every exponent
        rng.integers(1, 6 * 2 ** 20, 1024) * TINY,                           # subnormal quotients
        np.ldexp(1.0 + rng.random(256), rng.integers(-1074, -1019, 256)),    # near the boundary
        [np.inf, np.nan, 0.0, 1.7976931348623157e308, 6 * 2.0 ** -1022, 9 * TINY],
    ])
    s = np.concatenate([s, -s])
    u = np.zeros((len(s) + 2, 3, 3))
    u[1:-1, 1, 0] = s
    want = (s + 0.0) / 6.0     # the sum is s + 0 + 0 + 0 + 0 + 0 (-0 + 0 is +0)
    for method in ("plain", "tblock"):
        a = dev(u)
        out = jac.plain(a, torch.zeros_like(a), 1) if method == "plain" else \
            jac.tblock(a, torch.zeros_like(a), 1, t=1)
        torch.cuda.synchronize()
        got = out.cpu().numpy()[1:-1, 1, 1]
        if method == "plain":
            check_exact(got, want)
            continue
        q_ok = (want == 0) | (np.abs(want) >= 2.0 ** -1022)
        fin = np.isfinite(s)
        sel = q_ok & fin
        assert np.array_equal(bits(got[sel]), bits(want[sel]))
        assert np.all(np.isnan(got[~fin]))
        sub = fin & ~q_ok
        assert sub.any() and np.max(np.abs(got[sub] - want[sub])) <= TINY
