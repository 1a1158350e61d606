"""The allocation-free residual (jacobi_residual_f64_noalloc) against the
workspace entry point it varies (jacobi_residual_f64), through the C ABI:
the same r32 and norm bit for bit, on two calls in a row, the second on a
smaller grid (the fixed per-GPU array keeps the first call's partial sums),
and against the oracle's residual."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_0912_4506_amd import inputs

pytestmark = pytest.mark.gpu


def problem(nx, ny, nz, seed):
    x = inputs.laplace_problem(nx, ny, nz, seed=seed)
    x[1:-1, 1:-1, 1:-1] = inputs.grid(nx, ny, nz, seed=seed + 100)[1:-1, 1:-1, 1:-1]
    return x


def test_noalloc_residual_equals_workspace_residual(jac):
    for shape, seed in (((300, 170, 150), 1), ((40, 30, 20), 2)):
        x = problem(*shape, seed)
        xt = torch.from_numpy(x).to("cuda")
        r_ws = torch.zeros(xt.shape, dtype=torch.float32, device="cuda")
        n_ws = torch.zeros(1, dtype=torch.float64, device="cuda")
        jac.residual_f64(xt, r_ws, n_ws)
        r_na = torch.zeros_like(r_ws)
        n_na = torch.full_like(n_ws, float("nan"))
        jac.residual_f64_noalloc(xt, r_na, n_na)
        torch.cuda.synchronize()
        assert torch.equal(r_na, r_ws), shape
        assert n_na.item() == n_ws.item(), shape
        r_ref, n2_ref = oracle.residual(x)
        assert np.array_equal(r_na.cpu().numpy()[1:-1, 1:-1, 1:-1],
                              r_ref[1:-1, 1:-1, 1:-1].astype(np.float32))
        assert math.isclose(n_na.item(), n2_ref, rel_tol=1e-12)
