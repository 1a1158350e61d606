"""The bandwidth models against the values the paper prints
(tests/golden/paper_printed_values.txt, each line cited)."""
import os
from fractions import Fraction

import pytest

from paper_0912_4506_amd import perf_model as pm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_values.txt")


def records():
    out = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, args, value, cite = (f.strip() for f in line.split("|"))
        kw = dict(a.split("=") for a in args.split())
        out.append((name, {k: float(v) for k, v in kw.items()}, float(Fraction(value)), cite))
    return out



@pytest.mark.parametrize("name,kw,value,cite", records())
def test_printed_value(name, kw, value, cite):
    if name == "eq5_speedup":
        got = pm.speedup(kw["ms"], kw["ms1"], kw["mc"], kw["t"] * kw["T"])
        assert abs(got - value) <= 0.005 + 1e-12, cite          # printed to 2 decimals
    elif name == "eq5_closed_form":
        got = pm.speedup(kw["ms"], kw["ms1"], kw["mc"], kw["t"] * kw["T"])
        assert got == pytest.approx(value, rel=1e-14), cite
        assert pm.eq5_t4_closed_form(kw["T"]) == pytest.approx(value, rel=1e-14)
    elif name == "eq5_limit":
        assert pm.speedup_limit(kw["ms"], kw["mc"]) == value, cite
        assert pm.speedup(kw["ms"], 1.0, kw["mc"], 1e12) == pytest.approx(value, rel=1e-6)
    elif name == "mem_traffic":
        got = pm.memory_bandwidth_from_rate(kw["rate"], kw["fused"], int(kw["word"]))
        assert got == pytest.approx(value, rel=1e-12), cite
    elif name == "p0_printed":
        got = pm.p0(kw["ms"], int(kw["word"]))
        assert got == pytest.approx(value, rel=0.01), cite       # 2.3125 printed as 2.3
    else:
        raise AssertionError(f"unknown record {name}")


def test_block_time_consistent_with_speedup():
    """Eq. 5 is T0/Tb with T0 = tT * 16 B / M_s and Tb from Eq. 4."""
    ms, ms1, mc = 37e9, 10e9, 80e9
    for tT in (1, 2, 4, 8, 16):
        t0 = tT * 16.0 / ms
        assert t0 / pm.block_time(ms1, mc, tT) == pytest.approx(pm.speedup(ms, ms1, mc, tT), rel=1e-13)


def test_pass_planning_and_roofline():
    T = 100
    assert [pm.passes(T, t) for t in (1, 2, 4, 8, 16)] == [100, 50, 25, 13, 7]
    assert pm.t_eff(100, 8) == pytest.approx(100 / 13)
    assert pm.passes(0, 8) == 0
    assert pm.bytes_per_lup(8, 1) == 16 and pm.bytes_per_lup(4, 8) == 1.0
    assert pm.roofline(8e12, 100, 1) == pytest.approx(5e11)
    assert pm.roofline(8e12, 100, 4) == pytest.approx(2e12)
    assert pm.redundancy_overlapped(48, 48, 8) == pytest.approx((64 * 64) / (48 * 48))


@pytest.mark.parametrize("shape,tol,check,modes,seed,zero", [
    ((10, 9, 12), 1e-10, 1, 16, 0, True),    # every mode kept
    ((40, 33, 37), 1e-10, 1, 3, 0, True),    # truncated projection
    ((5, 1, 3), 1e-10, 1, 16, 0, True),      # a 1-cell axis
    ((12, 7, 9), 1e-9, 1, 2, 5, False),      # random initial interior
    ((12, 7, 9), 1e-9, 50, 2, 5, False),     # checked every 50 sweeps
])
def test_sweeps_to_tolerance_matches_oracle_solve(oracle_mod, shape, tol, check, modes, seed,
                                                  zero):
    """The spectral sweep count against a real Jacobi solve by the oracle,
    which checks its FP64 residual every ``check`` sweeps."""
    from paper_0912_4506_amd import inputs
    g = (inputs.laplace_problem if zero else inputs.grid)(*shape, seed=seed)
    _, sweeps, rel, ok = oracle_mod.jacobi_solve(g, tol, check_every=check)
    assert ok and rel <= tol
    got = pm.jacobi_sweeps_to_tolerance(g, tol, check_every=check, modes=modes)
    assert abs(got - sweeps) <= check


def test_sweeps_to_tolerance_single_mode():
    """Initial residual = one discrete sine mode: |r_s| = |lambda|^s |r_0|."""
    import math
    import numpy as np
    nx, ny, nz = 9, 6, 7
    a, b, c = 2, 1, 3
    i = np.arange(1, nx + 1)
    j = np.arange(1, ny + 1)
    k = np.arange(1, nz + 1)
    mode = (np.sin(math.pi * c * k / (nz + 1))[:, None, None]
            * np.sin(math.pi * b * j / (ny + 1))[None, :, None]
            * np.sin(math.pi * a * i / (nx + 1))[None, None, :])
    lam = (math.cos(math.pi * a / (nx + 1)) + math.cos(math.pi * b / (ny + 1))
           + math.cos(math.pi * c / (nz + 1))) / 3
    # x0 with zero shell and interior x: r0 = -(A x) = -(6 - 6 lam) x
    x0 = np.zeros((nz + 2, ny + 2, nx + 2))
    x0[1:-1, 1:-1, 1:-1] = mode
    tol = 1e-6
    want = math.ceil(math.log(tol) / math.log(abs(lam)) - 1e-9)
    assert pm.jacobi_sweeps_to_tolerance(x0, tol, modes=1) == want
    assert pm.jacobi_sweeps_to_tolerance(x0, tol, check_every=7) == -(-want // 7) * 7


def test_host_copy_bandwidth_is_a_sane_rate(oracle_mod):
    """The host copy probe behind the CPU baseline's P0 = M_s / 16 B: a
    positive, finite rate below any host's memory bandwidth, and -1 for a
    size or repeat count it cannot run."""
    import math
    ms = oracle_mod.copy_bandwidth(1 << 20, 3)
    assert math.isfinite(ms) and 1e8 < ms < 1e13
    assert oracle_mod._load().oracle_copy_bandwidth(0, 3, 1) == -1.0
    assert oracle_mod._load().oracle_copy_bandwidth(1 << 10, 0, 1) == -1.0
