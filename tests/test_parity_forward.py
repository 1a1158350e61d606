"""GPU parity of the forward sweeps (plain and temporally blocked) with the
CPU oracle, through the C ABI.

FP64: bitwise equality with the oracle (the kernels sum the six neighbours
in the printed order and divide by 6 with a correctly rounded quotient).
FP32: max |x32 - y64| <= 1e-5 where y64 is the FP64 oracle run on the FP32
inputs widened exactly (data uniform on [0, 1)).
"""
import numpy as np
import pytest
import torch

import oracle
from paper_0912_4506_amd import inputs

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5


def dev(u, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(u)).to("cuda", dtype)


def fits(bx, by, t):
    """A block has valid cells at depth t (halo t per side; i-halo even for
    blocks two cells per lane wide)."""
    hi = t + (t % 2) if bx % 128 == 0 else t
    return bx - 2 * hi >= 1 and by - 2 * t >= 1


def run_or_refused(jac, u, T, **kw):
    """The blocked result, or None when the library refuses the block for
    this depth (JAC_EUNSUPPORTED: too little LDS or no valid cells)."""
    from paper_0912_4506_amd._lib import JacobiError, JAC_EUNSUPPORTED
    try:
        return run(jac, u, T, **kw)
    except JacobiError as e:
        assert e.code == JAC_EUNSUPPORTED, e
        return None


def run(jac, u, T, method="tblock", dtype=torch.float64, **kw):
    a = dev(u, dtype)
    b = torch.full_like(a, float("nan"))   # b's prior contents must not matter
    out = jac.plain(a, b, T) if method == "plain" else jac.tblock(a, b, T, **kw)
    torch.cuda.synchronize()
    assert out.data_ptr() in (a.data_ptr(), b.data_ptr())
    return out.cpu().numpy().astype(np.float64)


def test_config0_plain_fp64_bitwise(jac):
    u = inputs.grid(64, 64, 64, seed=0)
    ref = oracle.sweeps(u, 10)
    got = run(jac, u, 10, "plain")
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("t", list(range(1, 9)))
def test_config0_tblock_fp64_bitwise_all_depths(jac, t):
    u = inputs.grid(64, 64, 64, seed=0)
    ref = oracle.sweeps(u, 10)
    for bx, by, w in jac.tile_menu(torch.float64):
        if not fits(bx, by, t):
            continue
        got = run_or_refused(jac, u, 10, t=t, bx=bx, by=by, waves=w)
        assert got is None or np.array_equal(got, ref), (t, bx, by, w)


@pytest.mark.parametrize("method,t", [("plain", None), ("tblock", 1), ("tblock", 4), ("tblock", 8)])
def test_config0_fp32(jac, method, t):
    u = inputs.grid(64, 64, 64, seed=0, dtype=np.float32)
    ref = oracle.sweeps(u.astype(np.float64), 10)
    got = run(jac, u, 10, method, dtype=torch.float32, t=t) if t else run(jac, u, 10, method,
                                                                           dtype=torch.float32)
    assert np.max(np.abs(got - ref)) <= FP32_TOL
    # shell bitwise
    m = np.ones(u.shape, bool)
    m[1:-1, 1:-1, 1:-1] = False
    assert np.array_equal(got[m], u.astype(np.float64)[m])


RAGGED = [((1, 1, 1), 3, 2, 0), ((3, 200, 2), 5, 3, 0), ((130, 33, 5), 11, 4, 2),
          ((127, 65, 70), 7, 8, 9), ((300, 31, 9), 9, 5, 1), ((241, 26, 13), 17, 6, 4),
          ((65, 97, 40), 16, 8, 0), ((2, 2, 100), 10, 7, 13)]


@pytest.mark.parametrize("shape,T,t,kchunk", RAGGED)
def test_ragged_shapes_bitwise(jac, shape, T, t, kchunk):
    """Shapes that leave ragged tails in i, j and k, several blocks per axis,
    T not a multiple of t, and explicit k-chunking."""
    nx, ny, nz = shape
    u = inputs.grid(nx, ny, nz, seed=hash(shape) % 1000)
    ref = oracle.sweeps(u, T)
    for bx, by, w in jac.tile_menu(torch.float64):
        if not fits(bx, by, t):
            continue
        got = run_or_refused(jac, u, T, t=t, bx=bx, by=by, kchunk=kchunk, waves=w)
        assert got is None or np.array_equal(got, ref), (shape, T, t, bx, by, w, kchunk)
    assert np.array_equal(run(jac, u, T, "plain"), ref)


def test_unsupported_depth_is_an_error(jac):
    """A block too small for the depth is refused (no kernel runs)."""
    from paper_0912_4506_amd._lib import JacobiError, JAC_EUNSUPPORTED
    u = inputs.grid(20, 20, 20, seed=1)
    for bx, by, w in jac.tile_menu(torch.float64):
        if not fits(bx, by, 8):
            with pytest.raises(JacobiError) as e:
                run(jac, u, 8, t=8, bx=bx, by=by, waves=w)
            assert e.value.code == JAC_EUNSUPPORTED


def test_padded_strides(jac):
    nx, ny, nz, T = 45, 37, 29, 9
    u = inputs.grid(nx, ny, nz, seed=5)
    ref = oracle.sweeps(u, T)
    big = torch.full((nz + 2, ny + 2 + 3, nx + 2 + 7), -1.0, dtype=torch.float64, device="cuda")
    for method in ("plain", "tblock"):
        a = big.clone()[:, :ny + 2, :nx + 2]
        a.copy_(dev(u))
        b = big.clone()[:, :ny + 2, :nx + 2]
        out = jac.plain(a, b, T) if method == "plain" else jac.tblock(a, b, T, t=4)
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), method


def test_out_idx_and_zero_sweeps(jac):
    u = inputs.grid(20, 10, 12, seed=1)
    a = dev(u)
    b = torch.zeros_like(a)
    assert jac.plain(a, b, 0).data_ptr() == a.data_ptr()
    assert jac.tblock(a, b, 0).data_ptr() == a.data_ptr()
    assert jac.plain(a, b, 1).data_ptr() == b.data_ptr()
    a = dev(u)
    # 9 sweeps at t=4: passes of depth 3, 3, 3 -> 3 passes -> result in b
    assert jac.tblock(a, torch.zeros_like(a), 9, t=4).data_ptr() != a.data_ptr()


@pytest.mark.parametrize("T,t", [(1, 1), (6, 3), (7, 4)])
def test_nan_cone(jac, T, t):
    """One interior NaN infects exactly the cells the oracle's does (compare
    isnan masks, not NaN payloads)."""
    nx, ny, nz = 140, 37, 20
    u = inputs.grid(nx, ny, nz, seed=3)
    u[10, 18, 120] = np.nan   # near the i-boundary of the first 128-wide block
    ref = oracle.sweeps(u, T)
    got = run(jac, u, T, t=t)
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    assert np.array_equal(got[~np.isnan(ref)], ref[~np.isnan(ref)])


def test_fp64_division_bitwise(jac):
    """The kernel's correctly rounded division against IEEE division on sums
    where multiplying by the rounded reciprocal is off by one ulp: a 1x1xN
    column whose shell faces carry the whole sum."""
    rng = np.random.default_rng(0)
    n = 4096
    s = rng.random(n) * 6.0
    s[: n // 2] = rng.integers(1, 2 ** 20, n // 2) / 1024.0
    u = np.zeros((n + 2, 3, 3))
    u[1:-1, 1, 0] = s            # i-1 face of cell (1, 1, k); every other neighbour 0
    got = run(jac, u, 1, t=1)
    assert np.array_equal(got[1:-1, 1, 1], s / 6.0)


def test_autotune_choice_is_used_and_exact(jac):
    """The autotuner returns a supported choice, the library then uses it for
    that geometry, and results stay bitwise."""
    nx, ny, nz, T = 90, 70, 60, 12
    u = inputs.grid(nx, ny, nz, seed=2)
    a = dev(u)
    b = torch.empty_like(a)
    (t, bx, by, w), ms = jac.autotune(a, b, T, tmax=6, reps=1)
    assert 1 <= t <= 6 and (bx, by, w) in jac.tile_menu(torch.float64) and ms > 0
    dt = jac.default_tile(a.shape, T)
    assert (dt[0], dt[1], dt[2], dt[4]) == (t, bx, by, w)
    a = dev(u)
    out = jac.tblock(a, torch.empty_like(a), T)
    assert np.array_equal(out.cpu().numpy(), oracle.sweeps(u, T))


def test_autotune_choice_survives_a_cache_file(jac, tmp_path):
    """A tuned choice, keyed by this device's architecture, written to a file,
    forgotten and read back: the library uses it again, bitwise."""
    nx, ny, nz, T = 70, 50, 40, 9
    u = inputs.grid(nx, ny, nz, seed=6)
    a = dev(u)
    (t, bx, by, w), _ = jac.autotune(a, torch.empty_like(a), T, tmax=4, reps=1)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    assert jac.tune_lookup(a, T) == (t, bx, by, 0, w)
    assert jac.tune_lookup(a, T, arch=arch) == (t, bx, by, 0, w)
    path = tmp_path / "tune.txt"
    jac.tune_save(path)
    assert f"{arch} f64 {nx} {ny} {nz} " in path.read_text()
    jac.tune_forget()
    assert jac.tune_lookup(a, T) is None
    assert jac.tune_load(path) >= 1
    assert jac.tune_lookup(a, T) == (t, bx, by, 0, w)
    dt = jac.default_tile(a.shape, T)
    assert (dt[0], dt[1], dt[2], dt[4]) == (t, bx, by, w)
    a = dev(u)
    out = jac.tblock(a, torch.empty_like(a), T)
    assert np.array_equal(out.cpu().numpy(), oracle.sweeps(u, T))
    jac.tune_forget()


def test_refused_tile_leaves_buffers_untouched(jac):
    """A block the library refuses at the requested depth is refused before
    anything is enqueued: a, b (and the adjoint's lam_a) keep their contents."""
    from paper_0912_4506_amd._lib import JacobiError, JAC_EUNSUPPORTED
    u = inputs.grid(40, 30, 20, seed=4)
    bad = [(bx, by, w) for bx, by, w in jac.tile_menu(torch.float64) if not fits(bx, by, 8)]
    assert bad
    for bx, by, w in bad:
        a = dev(u)
        b = torch.full_like(a, float("nan"))
        with pytest.raises(JacobiError) as e:
            jac.tblock(a, b, 16, t=8, bx=bx, by=by, waves=w)
        assert e.value.code == JAC_EUNSUPPORTED
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), u)
        assert bool(torch.isnan(b).all())
        with pytest.raises(JacobiError) as e:
            jac.adjoint(a, b, 16, t=8, bx=bx, by=by, waves=w)
        assert e.value.code == JAC_EUNSUPPORTED
        torch.cuda.synchronize()
        assert np.array_equal(a.cpu().numpy(), u)
        assert bool(torch.isnan(b).all())
