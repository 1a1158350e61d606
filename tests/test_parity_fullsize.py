"""GPU parity at the full workload sizes, in the launch configurations the
benchmark times, compared over the whole grid.

* 512^3 FP64, T = 100: the plain kernel, and the blocked pass at every depth
  the benchmark reports with the library's default block and with every
  block shape of the menu (the by-depth figures time each shape): bitwise,
  every cell, against
  the oracle's full run (about 2 s on the host).  The comparison runs on the
  GPU against an uploaded copy of the oracle's result.
* The same grid by the pipelined schedule (the best configuration, two with
  several passes in flight, and every setting of the looseness sweep) and in
  one array (the compressed grid) at the configurations the benchmark
  reports, bitwise; and in FP32 at
  the default blocking, every cell within 1e-5 of the FP64 oracle run on the
  FP32-rounded input.
* 768^3, the refinement's inner solve: 50 FP32 sweeps with a right-hand side
  at the library's default depth against the oracle's full FP64 run, and the
  FP64 residual and the fused update-and-residual bitwise over the whole grid.
"""
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


@pytest.fixture(scope="module")
def grid512():
    """(level-0 grid on the host, the oracle's level 100 on the GPU)."""
    u = inputs.grid(N, N, N, seed=0)
    ref = dev(oracle.sweeps(u, T))
    yield u, ref
    del ref
    torch.cuda.empty_cache()


def same_as(out, ref):
    """Bitwise equality of two float64 device tensors (no NaN in them)."""
    return bool(torch.equal(out.view(torch.int64), ref.view(torch.int64)))


def run_blocked(jac, u, **kw):
    a = dev(u)
    b = torch.full_like(a, float("nan"))
    out = jac.tblock(a, b, T, **kw)
    torch.cuda.synchronize()
    return out


def test_512_plain_full(jac, grid512):
    u, ref = grid512
    a = dev(u)
    b = torch.full_like(a, float("nan"))
    out = jac.plain(a, b, T)
    torch.cuda.synchronize()
    assert same_as(out, ref)


@pytest.mark.parametrize("t", [1, 2, 3, 4, 5, 6, 8])
def test_512_blocked_default_full(jac, grid512, t):
    """The benchmark's call: jacobi_tblock with the library's default block
    for depth t (t = 4 is the headline configuration), every cell."""
    u, ref = grid512
    assert same_as(run_blocked(jac, u, t=t), ref)


@pytest.mark.parametrize("t", [1, 2, 3, 4, 5, 6, 8])
def test_512_blocked_every_shape_full(jac, grid512, t):
    """Every block shape of the menu at every depth the benchmark's by-depth
    figures report (they time each shape and keep the fastest), every cell."""
    from paper_0912_4506_amd._lib import JacobiError, JAC_EUNSUPPORTED
    u, ref = grid512
    ran = 0
    for bx, by, w in jac.tile_menu(torch.float64):
        try:
            out = run_blocked(jac, u, t=t, bx=bx, by=by, waves=w)
        except JacobiError as e:
            assert e.code == JAC_EUNSUPPORTED, e
            continue
        assert same_as(out, ref), (t, bx, by, w)
        ran += 1
        del out
    assert ran >= (8 if t <= 6 else 2)


@pytest.mark.parametrize("team,t,kchunk", [(2, 4, 32), (1, 4, 128), (4, 2, 64)])
def test_512_pipelined_full(jac, grid512, team, t, kchunk):
    """The pipelined schedule at the workload size (the benchmark's best
    configuration, team 1, t = 4, 128-plane chunks, and two with several
    passes in flight), every cell."""
    u, ref = grid512
    a = dev(u)
    b = torch.full_like(a, float("nan"))
    plan = jac.PipelinePlan(a, b, T, team=team, t=t, kchunk=kchunk)
    plan.run("relaxed")
    torch.cuda.synchronize()
    assert not plan.wait_error()
    assert same_as(plan.results()[0], ref)


@pytest.mark.parametrize("team,t,kchunk", [(4, 1, 16), (8, 1, 32), (4, 2, 32), (4, 4, 64)])
def test_512_pipelined_looseness_full(jac, grid512, team, t, kchunk):
    """Every setting of the benchmark's looseness sweep (Eq. 3): lower
    distance 1 with upper distance 1 (lock step), 2, 4 and none, and upper
    distance 2 with a team delay of 8 chunks, each over the whole grid.  The
    waits change only the pacing: bitwise, and no wait gives up."""
    u, ref = grid512
    for du, dt in ((1, 0), (2, 0), (4, 0), (0, 0), (2, 8)):
        a = dev(u)
        b = torch.full_like(a, float("nan"))
        plan = jac.PipelinePlan(a, b, T, team=team, t=t, kchunk=kchunk, dl=1, du=du, dt=dt)
        plan.run("relaxed")
        torch.cuda.synchronize()
        assert not plan.wait_error(), (du, dt)
        assert same_as(plan.results()[0], ref), (du, dt)
        del a, b, plan


@pytest.mark.parametrize("t", [4, 5, 6])
def test_512_compressed_full(jac, grid512, t):
    """The compressed single grid at the workload size (the default block of
    each depth; t = 5 is the benchmark's best), every cell of the frame
    holding level T."""
    u, ref = grid512
    arr = torch.empty(jac.compressed_shape(N, N, N, t), dtype=torch.float64, device="cuda")
    jac.compressed_frame(arr, t, 0).copy_(torch.from_numpy(u))
    run = jac.Compressed(arr, T, t).run()
    torch.cuda.synchronize()
    assert not run.wait_error()
    res = run.result()
    assert bool(torch.equal(res, ref))
    del arr, run, res
    torch.cuda.empty_cache()


def test_512_fp32_blocked_default_full(jac):
    """FP32 at the workload size with the library's default blocking: every
    cell within 1e-5 of the FP64 oracle run on the FP32-rounded input."""
    u = inputs.grid(N, N, N, seed=0).astype(np.float32)
    ref = dev(oracle.sweeps(u.astype(np.float64), T))
    a = dev(u, torch.float32)
    b = torch.empty_like(a)
    out = jac.tblock(a, b, T)
    torch.cuda.synchronize()
    err = (out.double() - ref).abs().max().item()
    assert err <= 1e-5, err


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


def test_largest_planes_bitwise(jac):
    """Planes just under the 2 GiB the sweep kernels address with 32-bit
    byte offsets (15402^2 doubles = 1.90 GB per plane, 3 interior planes):
    the plain sweep and the blocked pass at its default blocking, every cell,
    bitwise against the oracle."""
    nx = ny = 15400
    nz, T = 3, 4
    assert (nx + 2) * (ny + 2) * 8 < 2 ** 31
    u = inputs.grid(nx, ny, nz, seed=7)
    ref = dev(oracle.sweeps(u, T))
    for method in ("plain", "tblock"):
        a = dev(u)
        b = torch.full_like(a, float("nan"))
        out = jac.plain(a, b, T) if method == "plain" else jac.tblock(a, b, T)
        torch.cuda.synchronize()
        assert same_as(out, ref), method
        del a, b, out
        torch.cuda.empty_cache()
