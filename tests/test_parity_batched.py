"""GPU parity of the batched runs (persistent with per-block counters, and
lockstep with one launch per pass) with the CPU oracle, and of their replay
from a captured graph."""
import numpy as np
import pytest
import torch

import oracle
from paper_0912_4506_amd import inputs

pytestmark = pytest.mark.gpu


def make_batch(shapes, seed=0, dtype=torch.float64):
    us = [inputs.batch_grid(s, m, seed=seed) for m, s in enumerate(shapes)]
    a = [torch.from_numpy(u).to("cuda", dtype) for u in us]
    b = [torch.full_like(x, float("nan")) for x in a]
    return us, a, b


SHAPES = [(32, 32, 32), (45, 17, 80), (130, 70, 33), (7, 200, 19), (1, 1, 1), (96, 96, 96),
          (61, 3, 129)]


@pytest.mark.parametrize("mode", ["relaxed", "lockstep"])
@pytest.mark.parametrize("t,tile", [(5, (64, 48)), (4, (128, 32)), (2, (64, 32)), (3, (64, 64))])
def test_batched_bitwise(jac, mode, t, tile):
    Ts = [50, 17, 23, 9, 4, 31, 12]
    us, a, b = make_batch(SHAPES)
    plan = jac.BatchPlan(a, b, Ts, t=t, bx=tile[0], by=tile[1])
    plan.run(mode)
    torch.cuda.synchronize()
    assert not plan.wait_error()
    for m, (u, T, out) in enumerate(zip(us, Ts, plan.results())):
        assert np.array_equal(out.cpu().numpy(), oracle.sweeps(u, T)), (m, mode, t, tile)


@pytest.mark.parametrize("mode", ["relaxed", "lockstep"])
@pytest.mark.parametrize("t,tile", [(3, (64, 64)), (5, (64, 60)), (8, (64, 48))])
def test_batched_full_depth_instance(jac, mode, t, tile):
    """Every T a multiple of t: every item has the full depth, and the run
    uses the kernel instance whose depth is a constant."""
    Ts = [t * q for q in (1, 4, 2, 7, 3, 5, 1)]
    us, a, b = make_batch(SHAPES, seed=9)
    plan = jac.BatchPlan(a, b, Ts, t=t, bx=tile[0], by=tile[1])
    plan.run(mode)
    torch.cuda.synchronize()
    assert not plan.wait_error()
    for m, (u, T, out) in enumerate(zip(us, Ts, plan.results())):
        assert np.array_equal(out.cpu().numpy(), oracle.sweeps(u, T)), (m, mode, t, tile)


def test_batched_small_kchunk(jac):
    """Several k chunks per grid: dependencies between chunks of one pass."""
    us, a, b = make_batch([(70, 50, 90), (33, 33, 40)])
    plan = jac.BatchPlan(a, b, [20, 13], t=4, bx=64, by=48, kchunk=8)
    plan.run("relaxed")
    torch.cuda.synchronize()
    for u, T, out in zip(us, [20, 13], plan.results()):
        assert np.array_equal(out.cpu().numpy(), oracle.sweeps(u, T))


def test_graph_replay(jac):
    """Capture the run once, replay it several times with eager work and
    synchronisations between replays; every replay matches the eager run."""
    us, a, b = make_batch(SHAPES[:4], seed=3)
    Ts = [20, 10, 15, 5]
    a0 = [x.clone() for x in a]
    plan = jac.BatchPlan(a, b, Ts, t=5, bx=64, by=48)
    plan.run("relaxed")
    torch.cuda.synchronize()
    eager = [x.clone() for x in plan.results()]
    for m in range(4):
        assert np.array_equal(eager[m].cpu().numpy(), oracle.sweeps(us[m], Ts[m]))
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for x, x0 in zip(a, a0):
            x.copy_(x0)
        plan.run("relaxed")  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.run("relaxed")
    for rep in range(4):
        for x, x0 in zip(a, a0):
            x.copy_(x0)
        for x in b:
            x.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for m, out in enumerate(plan.results()):
            assert torch.equal(out, eager[m]), (rep, m)


def test_batch_config_64_grids(jac):
    """The batched workload: 64 cubic grids, edges log-uniform in [32, 256],
    T = 50, FP64, one persistent launch; every grid bitwise vs the oracle."""
    edges = inputs.batch_edges(64, seed=0)
    us, a, b = make_batch(edges, seed=0)
    Ts = [50] * 64
    plan = jac.BatchPlan(a, b, Ts, t=5, bx=64, by=48)
    plan.run("relaxed")
    torch.cuda.synchronize()
    for m, (u, out) in enumerate(zip(us, plan.results())):
        assert np.array_equal(out.cpu().numpy(), oracle.sweeps(u, 50)), m


@pytest.mark.parametrize("case", range(12))
def test_batched_random_configs(jac, case):
    """Seeded random batches (shapes, sweep counts, depth, block shape, k
    chunk, FP32 or FP64) in relaxed mode, twice in a row on the same plan:
    the publication of finished blocks between workgroups (write-through
    stores, counters, acquire) must give the sequential result every time."""
    rng = np.random.default_rng(1000 + case)
    n = int(rng.integers(1, 9))
    shapes = [tuple(int(x) for x in rng.integers(1, 120, size=3)) for _ in range(n)]
    Ts = [int(x) for x in rng.integers(0, 30, size=n)]
    menu = jac.tile_menu(torch.float64)
    bx, by, w = menu[int(rng.integers(0, len(menu)))]
    t = int(rng.integers(1, 6))
    kc = int(rng.choice([0, 8, 16, 40]))
    dtype = torch.float64 if case % 3 else torch.float32
    us, a, b = make_batch(shapes, seed=case, dtype=dtype)
    try:
        plan = jac.BatchPlan(a, b, Ts, t=t, bx=bx, by=by, waves=w, kchunk=kc)
    except Exception as e:      # a block too small for the depth, or too little LDS
        from paper_0912_4506_amd._lib import JacobiError, JAC_EUNSUPPORTED
        assert isinstance(e, JacobiError) and e.code == JAC_EUNSUPPORTED, e
        pytest.skip(f"refused: {e}")
    refs = [oracle.sweeps(u.astype(np.float32).astype(np.float64) if dtype == torch.float32 else u, T)
            for u, T in zip(us, Ts)]
    for rep in range(2):
        if rep:
            for x, u in zip(a, us):
                x.copy_(torch.from_numpy(u).to("cuda", dtype))
        plan.run("relaxed")
        torch.cuda.synchronize()
        assert not plan.wait_error()
        for m, (ref, out) in enumerate(zip(refs, plan.results())):
            got = out.cpu().numpy().astype(np.float64)
            if dtype == torch.float64:
                assert np.array_equal(got, ref), (case, rep, m, shapes[m], Ts[m], t, bx, by, w, kc)
            else:
                assert np.max(np.abs(got - ref)) <= 1e-5, (case, rep, m)


@pytest.fixture(scope="module")
def batch64():
    """The batched workload (64 cubic grids, edges log-uniform in [32, 256],
    FP64, T = 50): level-0 grids on the host, the oracle's results on the GPU."""
    edges = inputs.batch_edges(64, seed=0)
    us = [inputs.batch_grid(e, m, seed=0) for m, e in enumerate(edges)]
    refs = [torch.from_numpy(oracle.sweeps(u, 50)).to("cuda") for u in us]
    yield us, refs
    del refs
    torch.cuda.empty_cache()


def test_batch_64_grids_every_autotune_candidate(jac, batch64):
    """Every (t, block) the batch autotuner can pick for the benchmark's
    workload (depths 2..6 times the menu; the benchmark times the pick, in a
    graph replay): one persistent launch each, every grid bitwise."""
    from paper_0912_4506_amd._lib import JacobiError, JAC_EUNSUPPORTED
    us, refs = batch64
    a = [torch.from_numpy(u).to("cuda") for u in us]
    a0 = [x.clone() for x in a]
    b = [torch.empty_like(x) for x in a]
    ran = 0
    for (bx, by, w) in jac.tile_menu(torch.float64):
        for t in range(2, 7):
            try:
                plan = jac.BatchPlan(a, b, [50] * 64, t=t, bx=bx, by=by, waves=w)
            except JacobiError as e:
                assert e.code == JAC_EUNSUPPORTED, e
                continue
            for x, x0 in zip(a, a0):
                x.copy_(x0)
            for x in b:
                x.fill_(float("nan"))
            plan.run("relaxed")
            torch.cuda.synchronize()
            assert not plan.wait_error(), (t, bx, by, w)
            for m, (ref, out) in enumerate(zip(refs, plan.results())):
                assert torch.equal(out, ref), (t, bx, by, w, m)
            ran += 1
    assert ran >= 20


def test_batch_64_grids_graph_replays_bench_pick(jac, batch64):
    """The benchmark's launch: depth 5, 64 x 64 blocks of 16 waves (the
    constant-depth instance, every T a multiple of t), captured in a graph
    and replayed three times; every replay of every grid bitwise."""
    us, refs = batch64
    a = [torch.from_numpy(u).to("cuda") for u in us]
    a0 = [x.clone() for x in a]
    b = [torch.empty_like(x) for x in a]
    plan = jac.BatchPlan(a, b, [50] * 64, t=5, bx=64, by=64, waves=16)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run("relaxed")
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.run("relaxed")
    for rep in range(3):
        for x, x0 in zip(a, a0):
            x.copy_(x0)
        for x in b:
            x.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert not plan.wait_error()
        for m, (ref, out) in enumerate(zip(refs, plan.results())):
            assert torch.equal(out, ref), (rep, m)


@pytest.mark.parametrize("mode", ["relaxed", "lockstep"])
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_batched_stress_bitwise(jac, mode, seed):
    """Race test of the per-block counters: the items of each pass shuffled
    and about a quarter of them held back by up to 8 sleep rounds before they
    start (jacobi_batched_stress), so consumers often reach a counter before
    its producer has started.  Results are bitwise those of the oracle and
    no wait gives up."""
    Ts = [20, 17, 23, 9, 4, 31, 12]
    us, a, b = make_batch(SHAPES, seed=seed)
    plan = jac.BatchPlan(a, b, Ts, t=3, bx=64, by=48, kchunk=16).stress(seed, 8)
    items = plan.items()
    assert any(d for *_, d in items)
    assert [p for _, p, _, _ in items] == sorted(p for _, p, _, _ in items)
    plan.run(mode)
    torch.cuda.synchronize()
    assert not plan.wait_error()
    for m, (u, T, out) in enumerate(zip(us, Ts, plan.results())):
        assert np.array_equal(out.cpu().numpy(), oracle.sweeps(u, T)), (m, mode, seed)


@pytest.mark.parametrize("mode", ["relaxed", "lockstep"])
def test_batched_zero_sweeps_and_single_cell(jac, mode):
    """A grid with T = 0 keeps its input (no items), a 1-cell grid and a grid
    thinner than a block run beside grids of many blocks."""
    shapes = [(40, 30, 20), (1, 1, 1), (9, 2, 70), (130, 70, 33)]
    Ts = [7, 5, 0, 12]
    us, a, b = make_batch(shapes, seed=4)
    plan = jac.BatchPlan(a, b, Ts, t=3, bx=64, by=48)
    plan.run(mode)
    torch.cuda.synchronize()
    assert not plan.wait_error()
    outs = plan.results()
    assert outs[2].data_ptr() == a[2].data_ptr()
    for m, (u, T, out) in enumerate(zip(us, Ts, outs)):
        assert np.array_equal(out.cpu().numpy(), oracle.sweeps(u, T) if T else u), (m, mode)
