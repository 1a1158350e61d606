"""GPU parity of the compressed single grid (jacobi_compressed) with the CPU
oracle: FP64 bitwise over the whole frame that holds level T (shell
included), FP32 within 1e-5, for several depths, remainder passes, k chunks,
block shapes and padded strides on ragged grids.  The array's cells outside
frame 0 start as NaN, so a read outside the input frame would show."""
import numpy as np
import pytest
import torch

import oracle
from paper_0912_4506_amd import inputs

pytestmark = pytest.mark.gpu


def layout(jac, u, t, dtype=torch.float64, pad=(0, 0)):
    """A compressed-grid array holding grid u (numpy) in frame 0."""
    nz, ny, nx = (s - 2 for s in u.shape)
    shp = jac.compressed_shape(nx, ny, nz, t)
    base = torch.full((shp[0], shp[1] + pad[0], shp[2] + pad[1]), float("nan"), dtype=dtype,
                      device="cuda")
    arr = base[:, :shp[1], :shp[2]]
    jac.compressed_frame(arr, t, 0).copy_(torch.from_numpy(np.ascontiguousarray(u)))
    return arr


@pytest.mark.parametrize("shape,T,t,kchunk,tile,pad", [
    ((70, 45, 33), 10, 4, 0, (0, 0, 0), (0, 0)),
    ((150, 100, 40), 9, 3, 8, (0, 0, 0), (0, 0)),
    ((130, 131, 29), 7, 2, 5, (64, 48, 8), (3, 5)),
    ((200, 70, 50), 13, 5, 12, (64, 56, 8), (0, 0)),
    ((96, 96, 64), 16, 8, 0, (0, 0, 0), (0, 0)),
    ((129, 77, 23), 5, 1, 4, (64, 72, 12), (0, 1)),
    ((300, 150, 37), 8, 4, 9, (64, 72, 12), (0, 0)),
    ((65, 1, 1), 3, 1, 0, (0, 0, 0), (0, 0)),
    ((1, 1, 1), 4, 2, 0, (0, 0, 0), (0, 0)),
    ((40, 50, 60), 2, 4, 0, (0, 0, 0), (0, 0)),
])
def test_compressed_fp64_bitwise(jac, shape, T, t, kchunk, tile, pad):
    u = inputs.grid(*shape, seed=11)
    ref = oracle.sweeps(u, T)
    bx, by, w = tile
    arr = layout(jac, u, t, pad=pad)
    run = jac.Compressed(arr, T, t, bx=bx, by=by, kchunk=kchunk, waves=w)
    for rep in range(2):        # a second run from the restored input: counters reset per run
        if rep:
            jac.compressed_frame(arr, t, 0).copy_(torch.from_numpy(u))
        run.run()
        torch.cuda.synchronize()
        assert not run.wait_error()
        assert run.frame == (-(-T // t)) % 2
        got = run.result().cpu().numpy()
        assert np.array_equal(got, ref)


def test_compressed_T0(jac):
    u = inputs.grid(30, 20, 10, seed=2)
    arr = layout(jac, u, 3)
    out = jac.compressed(arr, 0, 3)
    assert np.array_equal(out.cpu().numpy(), u)


def test_compressed_fp32(jac):
    u = inputs.grid(90, 61, 40, seed=8).astype(np.float32)
    ref = oracle.sweeps(u.astype(np.float64), 12)
    arr = layout(jac, u, 5, dtype=torch.float32)
    run = jac.Compressed(arr, 12, 5, kchunk=7).run()
    torch.cuda.synchronize()
    assert not run.wait_error()
    assert np.max(np.abs(run.result().cpu().numpy().astype(np.float64) - ref)) <= 1e-5


def test_compressed_matches_tblock(jac):
    """Same blocking as jacobi_tblock, one array instead of two: bitwise."""
    u = inputs.grid(160, 90, 70, seed=4)
    a = torch.from_numpy(u).cuda()
    b = torch.empty_like(a)
    want = jac.tblock(a, b, 20, t=4, bx=64, by=72, waves=12).cpu().numpy()
    arr = layout(jac, u, 4)
    got = jac.compressed(arr, 20, 4, bx=64, by=72, waves=12).cpu().numpy()
    assert np.array_equal(got, want)
