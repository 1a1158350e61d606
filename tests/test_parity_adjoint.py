"""GPU parity of the adjoint sweeps and the autograd wrappers with the CPU
oracle's adjoint (itself pinned to dense transposes, the dot-product identity
and finite differences on the CPU)."""
import numpy as np
import pytest
import torch

import oracle
from paper_0912_4506_amd import inputs

pytestmark = pytest.mark.gpu


def dev(u, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(u)).to("cuda", dtype)


def gpu_adjoint(jac, lam, T, dtype=torch.float64, **kw):
    a = dev(lam, dtype)
    b = torch.full_like(a, float("nan"))
    out = jac.adjoint(a, b, T, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("shape,T,t", [((16, 16, 16), 5, 2), ((33, 20, 17), 11, 4),
                                       ((70, 45, 31), 16, 8), ((1, 1, 1), 3, 1),
                                       ((2, 130, 3), 7, 3), ((131, 5, 66), 9, 5)])
def test_adjoint_fp64_bitwise(jac, shape, T, t):
    nx, ny, nz = shape
    lam = inputs.grid(nx, ny, nz, seed=7)
    ref = oracle.adjoint(lam, T)
    for bx, by, w in jac.tile_menu(torch.float64):
        hi = t + (t % 2) if bx % 128 == 0 else t
        if bx - 2 * hi < 1 or by - 2 * t < 1:
            continue
        from paper_0912_4506_amd._lib import JacobiError, JAC_EUNSUPPORTED
        try:
            got = gpu_adjoint(jac, lam, T, t=t, bx=bx, by=by, waves=w)
        except JacobiError as e:   # block refused at this depth (LDS)
            assert e.code == JAC_EUNSUPPORTED
            continue
        assert np.array_equal(got, ref), (shape, T, t, bx, by, w)


def test_adjoint_fp32(jac):
    nx, ny, nz, T = 40, 33, 28, 12
    lam = inputs.grid(nx, ny, nz, seed=8, dtype=np.float32)
    ref = oracle.adjoint(lam.astype(np.float64), T)
    got = gpu_adjoint(jac, lam, T, dtype=torch.float32, t=4)
    # the shell gradient sums up to T values in [0, 1): scale the bound by it
    assert np.max(np.abs(got - ref)) <= 1e-5 * max(1.0, T / 6.0)


def test_adjoint_zero_sweeps_is_identity(jac):
    lam = inputs.grid(10, 9, 8, seed=1)
    assert np.array_equal(gpu_adjoint(jac, lam, 0, t=2), lam)


def test_autograd_matches_oracle_and_fd(jac):
    """JacobiT: gradient of L = sum w * A_T^2 w.r.t. the whole input grid,
    against the oracle adjoint (bitwise) and central differences (FP64, 16^3;
    exact up to roundoff for a quadratic loss)."""
    from paper_0912_4506_amd.autograd import JacobiT
    nx = ny = nz = 16
    T, t = 12, 4
    u = inputs.grid(nx, ny, nz, seed=0)
    w = inputs.adjoint_weights(nx, ny, nz, seed=0)
    ut = dev(u).requires_grad_(True)
    wt = dev(w)
    A = JacobiT.apply(ut, T, t)
    L = (wt * A * A).sum()
    L.backward()
    g = ut.grad.cpu().numpy()
    ref = oracle.adjoint(2 * w * oracle.sweeps(u, T), T)
    assert np.array_equal(g, ref)

    def loss(v):
        a = torch.empty_like(v)
        out = jac.tblock(v.clone(), a, T, t=t)
        return float((wt * out * out).sum())

    rng = np.random.default_rng(1)
    cells = [tuple(int(x) for x in rng.integers(1, 17, 3)) for _ in range(5)]
    cells += [(0, 3, 4), (17, 5, 6), (4, 0, 9), (7, 17, 2), (8, 8, 0), (2, 3, 17), (0, 0, 5)]
    h = 1e-2
    gmax = np.max(np.abs(g))
    base = dev(u)
    for (i, j, k) in cells:
        up, dn = base.clone(), base.clone()
        up[k, j, i] += h
        dn[k, j, i] -= h
        fd = (loss(up) - loss(dn)) / (2 * h)
        assert abs(fd - g[k, j, i]) <= 1e-6 * gmax, (i, j, k, fd, g[k, j, i])


def test_checkpoints_gradients(jac):
    """Losses on intermediate checkpoints: the gradient equals the sum of the
    adjoints of each checkpoint's own loss."""
    from paper_0912_4506_amd.autograd import checkpoints
    nx, ny, nz, T, t = 18, 14, 12, 10, 4
    u = inputs.grid(nx, ny, nz, seed=3)
    ut = dev(u).requires_grad_(True)
    levels = checkpoints(ut, T, t)
    assert len(levels) == 3
    # the same checkpoints with a different kernel depth give the same forward levels
    lv2 = checkpoints(dev(u), T, t, depth=2)
    for x, y in zip(levels, lv2):
        assert torch.equal(x.detach(), y)
    w = [dev(inputs.adjoint_weights(nx, ny, nz, seed=s)) for s in range(3)]
    L = sum((wi * lv).sum() for wi, lv in zip(w, levels))
    L.backward()
    # the backward's order: the adjoint of the last segment, then the gradient
    # arriving at level 8 added (one rounding per element), and so on
    wn = [wi.cpu().numpy() for wi in w]
    horner = oracle.adjoint(oracle.adjoint(oracle.adjoint(wn[2], 2) + wn[1], 4) + wn[0], 4)
    assert np.array_equal(ut.grad.cpu().numpy(), horner)
    # and, by linearity, the sum of the adjoints of each checkpoint's own loss
    ref = sum(oracle.adjoint(wn[m], lv) for m, lv in enumerate((4, 8, 10)))
    assert np.max(np.abs(horner - ref)) <= 1e-13 * np.max(np.abs(ref))
    # forward values bitwise
    for lv, n in zip(levels, (4, 8, 10)):
        assert np.array_equal(lv.detach().cpu().numpy(), oracle.sweeps(u, n))


@pytest.mark.parametrize("t", [8, None])
def test_config_256_t32_fp64_bitwise(jac, t):
    """The differentiable workload's size: 256^3, T = 32, FP64, at t = 8 and
    at the library's default blocking (what the benchmark's autograd run
    uses)."""
    n, T = 256, 32
    lam = 2 * inputs.adjoint_weights(n, n, n, seed=0) * inputs.grid(n, n, n, seed=0)
    ref = oracle.adjoint(lam, T)
    got = gpu_adjoint(jac, lam, T, t=t)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("t", [8, None])
def test_config_256_t32_fp32(jac, t):
    """The differentiable workload in FP32: 256^3, T = 32, t = 8, against the
    oracle's FP64 adjoint of the FP32-rounded gradient.  The interior values
    are averages (bounded by the input's max); the shell gradient adds up to
    T of them, divided by 6."""
    n, T = 256, 32
    lam = (2 * inputs.adjoint_weights(n, n, n, seed=0) * inputs.grid(n, n, n, seed=0)).astype(np.float32)
    ref = oracle.adjoint(lam.astype(np.float64), T)
    got = gpu_adjoint(jac, lam, T, dtype=torch.float32, t=t)
    assert np.max(np.abs(got - ref)) <= 1e-5 * max(1.0, T / 6.0)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("T", [7, 32])
def test_default_tile_reports_the_adjoints_choice(jac, dtype, T):
    """default_tile(adjoint=True) names the blocking adjoint() takes when left
    to the library: the returned buffer follows the parity of ceil(T / t),
    and the result is bitwise that of the same blocking passed explicitly."""
    n = 70
    lam = 2 * inputs.adjoint_weights(n, n, n, seed=3) * inputs.grid(n, n, n, seed=3)
    t, bx, by, _, waves = jac.default_tile(lam.shape, T, dtype=dtype, adjoint=True)
    a = dev(lam, dtype)
    b = torch.zeros_like(a)
    out = jac.adjoint(a, b, T)
    assert out is (b if -(-T // t) % 2 else a)
    got = out.cpu().numpy()
    want = gpu_adjoint(jac, lam, T, dtype=dtype, t=t, bx=bx, by=by, waves=waves)
    assert np.array_equal(got.astype(np.float64), want)
