"""GPU parity of the D3Q19 lattice Boltzmann steps (lbm_d3q19_steps, through
the C ABI) with the CPU oracle (oracle/lbm.c, pinned by tests/test_oracle_lbm.py):
FP64 bitwise (the kernel keeps the oracle's order of operations), FP32
within 2e-6 of the FP64 oracle on the FP32-rounded input, on ragged boxes
and at the size the benchmark times."""
import numpy as np
import pytest
import torch

import oracle
from paper_0912_4506_amd import inputs

pytestmark = pytest.mark.gpu


def run(jac, f, omega, T, dtype=torch.float64):
    a = torch.from_numpy(np.ascontiguousarray(f)).to("cuda", dtype)
    b = torch.full_like(a, float("nan"))
    out = jac.lbm_d3q19(a, b, omega, T)
    torch.cuda.synchronize()
    assert out.data_ptr() == (b.data_ptr() if T % 2 else a.data_ptr())
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 5, 4), (64, 4, 3), (65, 33, 17), (130, 9, 12),
                                   (3, 70, 5)])
@pytest.mark.parametrize("omega,T", [(1.0, 1), (1.7, 6), (0.6, 5)])
def test_lbm_fp64_bitwise(jac, shape, omega, T):
    nx, ny, nz = shape
    f = inputs.lbm_populations(nx, ny, nz, seed=sum(shape))
    ref = oracle.lbm_d3q19(f, omega, T)
    assert np.array_equal(run(jac, f, omega, T), ref)


def test_lbm_fp32(jac):
    f = inputs.lbm_populations(70, 20, 9, seed=5).astype(np.float32)
    ref = oracle.lbm_d3q19(f.astype(np.float64), 1.3, 8)
    got = run(jac, f, 1.3, 8, torch.float32)
    assert np.max(np.abs(got - ref)) <= 2e-6 * np.max(np.abs(ref))


def test_lbm_zero_steps_and_streaming_only(jac):
    """T = 0 leaves f in place; omega = 0 streams only (an exact shift)."""
    f = inputs.lbm_populations(9, 6, 5, seed=6)
    assert np.array_equal(run(jac, f, 1.0, 0), f)
    assert np.array_equal(run(jac, f, 0.0, 3), oracle.lbm_d3q19(f, 0.0, 3))


def test_lbm_bench_size_bitwise(jac):
    """The benchmark's launch (256^3 box, FP64, omega = 1.7), four steps,
    every population of every cell against the oracle."""
    n = 256
    f = inputs.lbm_populations(n, n, n, seed=0)
    ref = torch.from_numpy(oracle.lbm_d3q19(f, 1.7, 4)).to("cuda")
    a = torch.from_numpy(f).to("cuda")
    b = torch.empty_like(a)
    out = jac.lbm_d3q19(a, b, 1.7, 4)
    torch.cuda.synchronize()
    assert bool(torch.equal(out.view(torch.int64), ref.view(torch.int64)))


def run_blocked(jac, f, omega, T, dtype=torch.float64, kchunk=0):
    a = torch.from_numpy(np.ascontiguousarray(f)).to("cuda", dtype)
    b = torch.full_like(a, float("nan"))
    out = jac.lbm_d3q19(a, b, omega, T, blocked=True, kchunk=kchunk)
    torch.cuda.synchronize()
    launches = T // 2 + T % 2
    assert out.data_ptr() == (b.data_ptr() if launches % 2 else a.data_ptr())
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("shape", [(1, 1, 1), (7, 5, 4), (30, 6, 8), (31, 7, 9), (65, 33, 17),
                                   (130, 9, 12), (3, 70, 5), (61, 13, 2)])
@pytest.mark.parametrize("omega,T,kchunk", [(1.0, 2, 0), (1.7, 6, 0), (0.6, 5, 3), (1.2, 1, 0),
                                            (1.5, 4, 1)])
def test_lbm_blocked_fp64_bitwise(jac, shape, omega, T, kchunk):
    """Two steps per pass (lbm_d3q19_blocked): ragged tiles along x and y
    (30 x 6 cells each), boxes smaller than a tile, several z chunks (kchunk
    1 and 3), odd T (a plain step at the end), against the oracle, bitwise."""
    nx, ny, nz = shape
    f = inputs.lbm_populations(nx, ny, nz, seed=sum(shape) + T)
    ref = oracle.lbm_d3q19(f, omega, T)
    assert np.array_equal(run_blocked(jac, f, omega, T, kchunk=kchunk), ref)


@pytest.mark.parametrize("shape,T,kchunk", [((70, 20, 9), 8, 0), ((1, 1, 1), 3, 0),
                                            ((30, 14, 5), 4, 0), ((31, 15, 9), 5, 3),
                                            ((65, 33, 17), 6, 0), ((7, 40, 6), 2, 1)])
def test_lbm_blocked_fp32_equals_plain(jac, shape, T, kchunk):
    """FP32 (32 x 16 regions, 30 x 14 output tiles): every cell runs the plain
    kernel's instruction sequence, so the blocked passes equal the plain
    steps bitwise (and the oracle within the FP32 bound)."""
    f = inputs.lbm_populations(*shape, seed=5 + T).astype(np.float32)
    got = run_blocked(jac, f, 1.3, T, torch.float32, kchunk=kchunk)
    plain = run(jac, f, 1.3, T, torch.float32)
    assert np.array_equal(got, plain)
    ref = oracle.lbm_d3q19(f.astype(np.float64), 1.3, T)
    assert np.max(np.abs(got - ref)) <= 2e-6 * T * np.max(np.abs(ref))


def test_lbm_blocked_bench_size_bitwise(jac):
    """The benchmark's blocked launch (256^3, FP64, omega = 1.7, default z
    chunks): four steps in two passes, every value against the oracle."""
    n = 256
    f = inputs.lbm_populations(n, n, n, seed=0)
    ref = torch.from_numpy(oracle.lbm_d3q19(f, 1.7, 4)).to("cuda")
    a = torch.from_numpy(f).to("cuda")
    b = torch.empty_like(a)
    out = jac.lbm_d3q19(a, b, 1.7, 4, blocked=True)
    torch.cuda.synchronize()
    assert out.data_ptr() == a.data_ptr()
    assert bool(torch.equal(out.view(torch.int64), ref.view(torch.int64)))
