"""GPU parity of pipelined temporal blocking (jacobi_pipelined_plan run by
jacobi_batched_run in relaxed mode) with the CPU oracle: FP64 bitwise, FP32
within 1e-5, for several team sizes, sweeps per item, k chunks and block
shapes on ragged grids, and for several settings of the relaxed
synchronisation of Eq. 3 (lower distance, upper distance, team delay)."""
import numpy as np
import pytest
import torch

import oracle
from paper_0912_4506_amd import inputs

pytestmark = pytest.mark.gpu


def dev(u, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(u)).to("cuda", dtype)


@pytest.mark.parametrize("shape,T,team,t,kchunk,tile", [
    ((130, 70, 64), 13, 4, 1, 16, (0, 0, 0)),
    ((130, 70, 64), 13, 1, 2, 8, (0, 0, 0)),
    ((130, 70, 64), 20, 7, 1, 4, (64, 56, 8)),
    ((70, 45, 33), 9, 3, 3, 5, (64, 72, 12)),
    ((70, 45, 33), 9, 100, 1, 16, (64, 64, 16)),
    ((200, 151, 97), 11, 5, 2, 12, (64, 48, 8)),
])
def test_pipelined_fp64_bitwise(jac, shape, T, team, t, kchunk, tile):
    u = inputs.grid(*shape, seed=7)
    ref = oracle.sweeps(u, T)
    a = dev(u)
    b = torch.full_like(a, float("nan"))
    bx, by, w = tile
    plan = jac.PipelinePlan(a, b, T, team=team, t=t, bx=bx, by=by, kchunk=kchunk, waves=w)
    for rep in range(2):        # a second run from the restored input: counters reset per run
        if rep:
            a.copy_(dev(u))
            b.fill_(float("nan"))
        plan.run("relaxed")
        torch.cuda.synchronize()
        assert not plan.wait_error()
        assert np.array_equal(plan.results()[0].cpu().numpy(), ref)


def test_pipelined_fp32(jac):
    u = inputs.grid(90, 61, 40, seed=8).astype(np.float32)
    ref = oracle.sweeps(u.astype(np.float64), 12)
    a = dev(u, torch.float32)
    b = torch.empty_like(a)
    out = jac.pipelined(a, b, 12, team=3, t=2, kchunk=8)
    torch.cuda.synchronize()
    assert np.max(np.abs(out.cpu().numpy().astype(np.float64) - ref)) <= 1e-5


def test_pipelined_lockstep_refused(jac):
    from paper_0912_4506_amd._lib import JacobiError
    a = dev(inputs.grid(20, 20, 20, seed=1))
    plan = jac.PipelinePlan(a, torch.empty_like(a), 4, team=2)
    with pytest.raises(JacobiError):
        plan.run("lockstep")


@pytest.mark.parametrize("sync", [(1, 1, 0), (1, 2, 0), (1, 4, 0), (2, 3, 0), (1, 2, 8), (3, 0, 2)])
@pytest.mark.parametrize("shape,T,team,t,kchunk", [
    ((130, 70, 200), 17, 4, 1, 8),
    ((70, 45, 97), 12, 3, 2, 6),
])
def test_pipelined_relaxed_sync_bitwise(jac, shape, T, team, t, kchunk, sync):
    """Lock-step (dl = du = 1), loose pipelines (du = 2, 4), a wider lower
    distance, a team delay: the waits change the pacing only, so every
    result is bitwise the oracle's, on two runs of one plan."""
    dl, du, dt = sync
    u = inputs.grid(*shape, seed=11)
    ref = oracle.sweeps(u, T)
    a = dev(u)
    b = torch.full_like(a, float("nan"))
    plan = jac.PipelinePlan(a, b, T, team=team, t=t, kchunk=kchunk, dl=dl, du=du, dt=dt)
    for rep in range(2):
        if rep:
            a.copy_(dev(u))
            b.fill_(float("nan"))
        plan.run("relaxed")
        torch.cuda.synchronize()
        assert not plan.wait_error(), (sync, rep)
        assert np.array_equal(plan.results()[0].cpu().numpy(), ref), (sync, rep)


@pytest.mark.parametrize("sync,seed", [((1, 1, 0), 5), ((1, 2, 0), 6), ((2, 3, 1), 7)])
def test_pipelined_stress_bitwise(jac, sync, seed):
    """The pipelined order with about a quarter of the items held back by up
    to 16 sleep rounds before they start: the Eq. 3 waits absorb the delays
    and the result stays bitwise the oracle's."""
    dl, du, dt = sync
    shape, T = (130, 70, 120), 12
    u = inputs.grid(*shape, seed=seed)
    a = dev(u)
    b = torch.full_like(a, float("nan"))
    plan = jac.PipelinePlan(a, b, T, team=4, t=1, kchunk=8, dl=dl, du=du, dt=dt).stress(seed, 16)
    plan.run("relaxed")
    torch.cuda.synchronize()
    assert not plan.wait_error(), sync
    assert np.array_equal(plan.results()[0].cpu().numpy(), oracle.sweeps(u, T)), sync
