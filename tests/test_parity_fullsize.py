"""GPU parity at the full workload sizes, in the launch configurations the
benchmark times.

* 512^3 FP64, T = 100: the plain kernel and the blocked pass at every depth
  the benchmark reports (the library's default block for each), compared
  bitwise with the oracle at sampled cells, which the oracle computes one by
  one from their domain of dependence.  The samples include the shell
  corners, the edges of the blocks and k chunks the default plan uses, and
  random interior cells.
* The same 512^3 grid by the pipelined schedule and in one array (the
  compressed grid), bitwise, and in FP32 at the default blocking (within 1e-5
  of the oracle on the FP32-rounded input).
* 768^3, the refinement's inner solve: 50 FP32 sweeps with a right-hand side
  at the library's default depth against the oracle's full FP64 run, and the
  FP64 residual and the fused update-and-residual bitwise over the whole grid.
"""
import concurrent.futures as cf
import math

import numpy as np
import pytest
import torch

import oracle
from paper_0912_4506_amd import inputs

pytestmark = pytest.mark.gpu

N, T = 512, 100


def dev(u, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(u)).to("cuda", dtype)


def samples():
    """(i, j, k) array indices of the sampled cells."""
    rng = np.random.default_rng(123)
    pts = {(1, 1, 1), (N, N, N), (1, N, 1), (N, 1, N), (N // 2, N // 2, N // 2)}
    # block edges at depth 4: 64-lane blocks start their valid i ranges at 1,
    # 60, 116, ..., 508; 72-row blocks (the default) their j ranges at 1, 68,
    # 132, ..., 452, and 56-row blocks at 1, 52, 100, ..., 484; k chunks of
    # 2, 3 or 5 per column meet near 257, 172 / 343 and 103 / 206 / ...
    for i in (59, 60, 115, 116, 507, 508):
        pts.add((i, int(rng.integers(1, N + 1)), int(rng.integers(1, N + 1))))
    for j in (67, 68, 131, 132, 451, 452, 51, 52, 483, 484):
        pts.add((int(rng.integers(1, N + 1)), j, int(rng.integers(1, N + 1))))
    for k in (256, 257, 171, 172, 342, 343, 103, 104, 2, N - 1):
        pts.add((int(rng.integers(1, N + 1)), int(rng.integers(1, N + 1)), k))
    while len(pts) < 48:
        pts.add(tuple(int(x) for x in rng.integers(1, N + 1, size=3)))
    return sorted(pts)


@pytest.fixture(scope="module")
def grid512():
    u = inputs.grid(N, N, N, seed=0)
    pts = samples()
    with cf.ThreadPoolExecutor(max_workers=16) as ex:
        ref = list(ex.map(lambda p: oracle.point(u, T, *p), pts))
    return u, pts, np.array(ref)


def sampled(out, pts):
    h = out.cpu().numpy()
    return np.array([h[k, j, i] for i, j, k in pts])


def test_512_plain_sampled(jac, grid512):
    u, pts, ref = grid512
    a = dev(u)
    b = torch.full_like(a, float("nan"))
    out = jac.plain(a, b, T)
    torch.cuda.synchronize()
    assert np.array_equal(sampled(out, pts), ref)


@pytest.mark.parametrize("t", [1, 2, 3, 4, 5, 6, 8])
def test_512_blocked_default_sampled(jac, grid512, t):
    """The benchmark's call: jacobi_tblock with the library's default block
    for depth t (t = 4 is the headline configuration)."""
    u, pts, ref = grid512
    a = dev(u)
    b = torch.full_like(a, float("nan"))
    out = jac.tblock(a, b, T, t=t)
    torch.cuda.synchronize()
    got = sampled(out, pts)
    bad = [(p, g, r) for p, g, r in zip(pts, got, ref) if not g == r]
    assert not bad, bad[:5]


def test_512_pipelined_sampled(jac, grid512):
    """The pipelined schedule at the workload size (two passes in flight,
    4 sweeps per item, 32-plane chunks), bitwise at the sampled cells."""
    u, pts, ref = grid512
    a = dev(u)
    b = torch.full_like(a, float("nan"))
    out = jac.pipelined(a, b, T, team=2, t=4, kchunk=32)
    torch.cuda.synchronize()
    assert np.array_equal(sampled(out, pts), ref)


def test_512_compressed_sampled(jac, grid512):
    """The compressed single grid at the workload size (t = 4, the default
    block), bitwise at the sampled cells of the frame holding level T."""
    u, pts, ref = grid512
    arr = torch.empty(jac.compressed_shape(N, N, N, 4), dtype=torch.float64, device="cuda")
    jac.compressed_frame(arr, 4, 0).copy_(torch.from_numpy(u))
    run = jac.Compressed(arr, T, 4).run()
    torch.cuda.synchronize()
    assert not run.wait_error()
    assert np.array_equal(sampled(run.result(), pts), ref)


@pytest.fixture(scope="module")
def grid512_f32():
    u = inputs.grid(N, N, N, seed=0).astype(np.float32).astype(np.float64)
    pts = samples()[::3]
    with cf.ThreadPoolExecutor(max_workers=16) as ex:
        ref = list(ex.map(lambda p: oracle.point(u, T, *p), pts))
    return u, pts, np.array(ref)


def test_512_fp32_blocked_default_sampled(jac, grid512_f32):
    """FP32 at the workload size with the library's default blocking: within
    1e-5 of the FP64 oracle run on the FP32-rounded input."""
    u, pts, ref = grid512_f32
    a = dev(u, torch.float32)
    b = torch.empty_like(a)
    out = jac.tblock(a, b, T)
    torch.cuda.synchronize()
    assert np.max(np.abs(sampled(out, pts).astype(np.float64) - ref)) <= 1e-5


def test_768_rhs_fp32_default(jac):
    """The inner solve of the 768^3 refinement at its default blocking (50
    FP32 sweeps, zero guess, right-hand side r) against the oracle in FP64 on
    the same (FP32-rounded) r: within 1e-5 of max|e|."""
    n, sweeps = 768, 50
    r = inputs.grid(n, n, n, seed=1).astype(np.float32)
    ref = oracle.rhs_sweeps(r.astype(np.float64), sweeps)
    a = torch.zeros(r.shape, dtype=torch.float32, device="cuda")
    b = torch.full_like(a, float("nan"))
    out = jac.tblock(a, b, sweeps, rhs=dev(r, torch.float32))
    got = out.cpu().numpy()
    err = np.max(np.abs(got.astype(np.float64) - ref))
    assert err <= 1e-5 * np.max(np.abs(ref)), err


def test_768_residual_and_fused_update(jac):
    """The FP64 residual and the fused update-and-residual over the whole
    768^3 grid, bitwise before the cast to float; norms to 1e-12."""
    n = 768
    x = inputs.laplace_problem(n, n, n, seed=0)
    x[1:-1, 1:-1, 1:-1] = inputs.grid(n, n, n, seed=5)[1:-1, 1:-1, 1:-1]
    e = np.zeros(x.shape, dtype=np.float32)
    e[1:-1, 1:-1, 1:-1] = inputs.grid(n, n, n, seed=6, dtype=np.float32)[1:-1, 1:-1, 1:-1] - 0.5
    xt, et = dev(x), dev(e, torch.float32)
    r32 = torch.zeros(xt.shape, dtype=torch.float32, device="cuda")
    norm2 = torch.zeros(1, dtype=torch.float64, device="cuda")
    jac.residual_f64(xt, r32, norm2)
    r_ref, n2_ref = oracle.residual(x)
    assert np.array_equal(r32.cpu().numpy()[1:-1, 1:-1, 1:-1],
                          r_ref[1:-1, 1:-1, 1:-1].astype(np.float32))
    assert math.isclose(norm2.item(), n2_ref, rel_tol=1e-12)
    del r_ref
    xn = xt.clone()
    z = torch.ones_like(r32)
    jac.update_residual_f64(xt, et, xn, r32, z, norm2)
    want = x
    want[1:-1, 1:-1, 1:-1] += e[1:-1, 1:-1, 1:-1].astype(np.float64)
    assert np.array_equal(xn.cpu().numpy(), want)
    r_ref, n2_ref = oracle.residual(want)
    assert np.array_equal(r32.cpu().numpy()[1:-1, 1:-1, 1:-1],
                          r_ref[1:-1, 1:-1, 1:-1].astype(np.float32))
    assert math.isclose(norm2.item(), n2_ref, rel_tol=1e-12)
    assert torch.count_nonzero(z[1:-1, 1:-1, 1:-1]).item() == 0
