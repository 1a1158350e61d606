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
