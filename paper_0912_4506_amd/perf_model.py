"""Bandwidth models for Jacobi sweeps (Sect. 1.1 and Sect. 1.4 of the paper).

All bandwidths in bytes/s, rates in lattice-site updates per second (LUP/s).
A "word" is 8 bytes for FP64 and 4 for FP32.  The paper counts one read and
one write per cell update once spatial blocking and non-temporal stores remove
the third word (read for ownership), hence 16 bytes per update in FP64.
"""
import math

import numpy as np


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


def _sine_modes(n, idx):
    """Orthonormal eigenvectors of the 1-D Dirichlet chain of n cells
    (discrete sine basis), columns for the wave numbers in idx."""
    i = np.arange(1, n + 1, dtype=np.float64)[:, None]
    return math.sqrt(2.0 / (n + 1)) * np.sin(np.pi * i * np.asarray(idx, np.float64)[None, :] / (n + 1))


def _kept_modes(n, k):
    """Wave numbers 1..k and n-k+1..n (all of 1..n when they overlap)."""
    if 2 * k >= n:
        return np.arange(1, n + 1)
    return np.concatenate([np.arange(1, k + 1), np.arange(n - k + 1, n + 1)])


def jacobi_sweeps_to_tolerance(x0, tol, check_every=1, modes=16):
    """Jacobi sweeps (the update of Sect. 1.1) needed to bring the residual
    r = (six neighbours) - 6x of the Dirichlet problem on grid x0 (shell =
    boundary data, interior = initial guess) to |r_s| <= tol |r_0|, rounded up
    to a multiple of ``check_every`` (the solve checks only then).

    One sweep maps the residual to r_{s+1} = J r_s with J = adjacency / 6, whose
    eigenvectors are products of discrete sines and whose eigenvalues are
    (cos(pi a/(nx+1)) + cos(pi b/(ny+1)) + cos(pi c/(nz+1))) / 3.  So
    |r_s|^2 = sum over modes of c^2 lambda^(2s), with c the projections of r_0.
    Only the ``modes`` lowest and highest wave numbers per axis are projected
    (|lambda| is largest there); the energy of the others is bounded by their
    largest |lambda|, and ``modes`` doubles until that bound cannot move the
    answer.  Exact arithmetic: a real solve may stop one sweep either side
    when its residual lands within rounding of the threshold."""
    x0 = np.asarray(x0, dtype=np.float64)
    nz, ny, nx = (d - 2 for d in x0.shape)
    if min(nx, ny, nz) < 1 or not tol > 0 or check_every < 1:
        raise ValueError("need a grid with an interior, tol > 0 and check_every >= 1")
    r = x0[1:-1, 1:-1, 1:-1] * -6.0
    r += x0[1:-1, 1:-1, :-2]
    r += x0[1:-1, 1:-1, 2:]
    r += x0[1:-1, :-2, 1:-1]
    r += x0[1:-1, 2:, 1:-1]
    r += x0[:-2, 1:-1, 1:-1]
    r += x0[2:, 1:-1, 1:-1]
    total = float(np.vdot(r, r))
    if total == 0.0:
        return 0
    target = tol * tol * total
    ns = (nx, ny, nz)
    while True:
        idx = [_kept_modes(n, modes) for n in ns]
        phi = [_sine_modes(n, i) for n, i in zip(ns, idx)]
        c = np.tensordot(r, phi[0], axes=([2], [0]))          # (z, y, a)
        c = np.tensordot(c, phi[1], axes=([1], [0]))          # (z, a, b)
        c = np.tensordot(c, phi[2], axes=([0], [0]))          # (a, b, c)
        cos = [np.cos(np.pi * i / (n + 1)) for n, i in zip(ns, idx)]
        lam = (cos[0][:, None, None] + cos[1][None, :, None] + cos[2][None, None, :]) / 3.0
        c2 = (c * c).ravel()
        lam2 = (lam * lam).ravel()
        kept = min(float(c2.sum()), total)
        lam_omit = 0.0
        c1 = [math.cos(math.pi / (n + 1)) for n in ns]
        for ax, n in enumerate(ns):
            if 2 * modes < n:
                lam_omit = max(lam_omit, abs(math.cos(math.pi * (modes + 1) / (n + 1))
                                             + sum(c1) - c1[ax]) / 3.0)
        omit = total - kept

        def f(s, extra):
            if s == 0:
                return total
            with np.errstate(divide="ignore"):
                v = float(np.sum(c2 * np.exp(s * np.log(lam2))))
            return v + (omit * lam_omit ** (2 * s) if extra else 0.0)

        def first(extra):
            hi = 1
            while f(hi, extra) > target:
                hi *= 2
            lo = hi // 2
            while hi - lo > 1:
                mid = (lo + hi) // 2
                if f(mid, extra) > target:
                    lo = mid
                else:
                    hi = mid
            return hi if f(lo, extra) > target else lo

        s_lo, s_hi = first(False), first(True)
        if s_lo == s_hi or all(2 * modes >= n for n in ns):
            return -(-s_lo // check_every) * check_every
        modes *= 2


__all__ = [n for n in dir() if not n.startswith("_") and n not in ("math", "np")]
