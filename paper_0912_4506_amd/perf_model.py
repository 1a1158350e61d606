"""Bandwidth models for Jacobi sweeps (Sect. 1.1 and Sect. 1.4 of the paper).

All bandwidths in bytes/s, rates in lattice-site updates per second (LUP/s).
A "word" is 8 bytes for FP64 and 4 for FP32.  The paper counts one read and
one write per cell update once spatial blocking and non-temporal stores remove
the third word (read for ownership), hence 16 bytes per update in FP64.
"""
import math


def bytes_per_lup(word=8, fused=1):
    """Memory traffic per update when ``fused`` sweeps share one memory pass:
    one word in and one word out per cell and pass (Sect. 1.1, code balance)."""
    return 2.0 * word / fused


def p0(ms, word=8):
    """Memory-bound baseline performance P0 = M_s / 16 B (Eq. 2), with M_s the
    copy bandwidth; ``word`` generalises the 16 B to 2 words."""
    return ms / bytes_per_lup(word, 1)


def passes(T, t):
    """HBM passes for T sweeps at blocking depth t: ceil(T/t) (the last pass
    takes the remainder)."""
    if T < 0 or t < 1:
        raise ValueError("need T >= 0 and t >= 1")
    return -(-T // t)


def t_eff(T, t):
    """Sweeps per memory pass averaged over the run: T / ceil(T/t)."""
    p = passes(T, t)
    return T / p if p else float(t)


def roofline(ms, T, t, word=8):
    """Memory roofline for T sweeps at depth t: M_s * t_eff / (2 words)."""
    return ms * t_eff(T, t) / bytes_per_lup(word, 1)


def memory_bandwidth_from_rate(rate_lups, fused, word=8):
    """Main-memory traffic implied by an update rate when ``fused`` updates
    share each transfer (the accounting used in the results of Sect. 1.5)."""
    return rate_lups * bytes_per_lup(word, fused)


def block_time(ms1, mc, tT, word=8):
    """Time for the tT updates a team applies to one cell's worth of data,
    Eq. 4: 16 B / M_s,1 + 2 (tT - 1) * 8 B / M_c."""
    return 2.0 * word / ms1 + 2.0 * (tT - 1) * word / mc


def speedup(ms, ms1, mc, tT):
    """Expected speedup of pipelined temporal blocking over the standard
    sweep, Eq. 5: (M_s,1 / M_s) * tT / (1 + (tT - 1) M_s,1 / M_c)."""
    return (ms1 / ms) * tT / (1.0 + (tT - 1) * ms1 / mc)


def speedup_limit(ms, mc):
    """Large-tT limit of Eq. 5: M_c / M_s."""
    return mc / ms


def alu_roof(flops_per_s, ops_per_lup, redundancy=1.0):
    """Update rate a kernel reaches when bound by arithmetic: issue rate over
    the operations each interior update costs (halo recomputation included
    through ``redundancy``)."""
    return flops_per_s / (ops_per_lup * redundancy)


def redundancy_overlapped(bx, by, t):
    """Cells computed per valid cell by an overlapped (trapezoid) tile of
    bx x by outputs that recomputes a halo shrinking by one per level, with
    every level computed over the full (bx+2t) x (by+2t) footprint."""
    return (bx + 2 * t) * (by + 2 * t) / float(bx * by)


def read_amplification(bx, by, t):
    """Level-0 cells read per output cell for an overlapped tile."""
    return (bx + 2 * t) * (by + 2 * t) / float(bx * by)


def eq5_t4_closed_form(T):
    """The paper's closed form at t = 4, M_s/M_s,1 = 2, M_c/M_s,1 = 8:
    16T / (7 + 4T)."""
    return 16.0 * T / (7.0 + 4.0 * T)


__all__ = [n for n in dir() if not n.startswith("_") and n != "math"]
