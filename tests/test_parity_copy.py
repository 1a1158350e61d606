"""GPU check of the copy kernel that measures M_s (Eq. 2): it moves every
byte of the range, exactly, and nothing past it."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes", [16, 4096 + 16, (1 << 20) * 37 + 48, 1 << 31])
def test_copy_moves_every_byte(jac, nbytes):
    g = torch.Generator(device="cuda").manual_seed(nbytes % 1000)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device="cuda", generator=g)
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda")
    jac.copy(dst[:nbytes], src)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src)
    assert int(dst[nbytes:].count_nonzero()) == 0


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("shape", [(7, 5, 3), (300, 9, 4), (257, 33, 17)])
def test_grid_add_every_element(jac, dtype, shape):
    """jacobi_grid_add: dst + src, one rounding per element, over the whole
    array (shell included): dense (flat kernel; element counts that are not
    a multiple of the 16-byte vector) and with padded strides (row kernel;
    the padding is left alone).  Compared with numpy's addition."""
    import numpy as np
    from paper_0912_4506_amd import inputs
    nx, ny, nz = shape
    npdt = np.float64 if dtype == torch.float64 else np.float32
    a = inputs.grid(nx, ny, nz, seed=1).astype(npdt)
    b = (inputs.grid(nx, ny, nz, seed=2) - 0.5).astype(a.dtype)
    dst = torch.from_numpy(a).cuda()
    jac.grid_add(dst, torch.from_numpy(b).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(dst.cpu().numpy(), a + b)
    big = torch.full((nz + 2, ny + 2 + 2, nx + 2 + 5), 7.0, dtype=dtype, device="cuda")
    d2 = big.clone()[:, :ny + 2, :nx + 2]
    s2 = big.clone()[:, :ny + 2, :nx + 2]
    d2.copy_(torch.from_numpy(a))
    s2.copy_(torch.from_numpy(b))
    jac.grid_add(d2, s2)
    torch.cuda.synchronize()
    assert np.array_equal(d2.cpu().numpy(), a + b)
    base = d2
    while base._base is not None:
        base = base._base
    full = base.cpu().numpy()
    assert np.all(full[:, ny + 2:, :] == 7.0) and np.all(full[:, :, nx + 2:] == 7.0)
    # dst == src doubles every element
    jac.grid_add(dst, dst)
    torch.cuda.synchronize()
    assert np.array_equal(dst.cpu().numpy(), 2 * (a + b))
