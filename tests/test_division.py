"""The three-operation FP64 division of the blocked kernels, emulated exactly
on the CPU (rational arithmetic, one rounding per operation, as the FMA
instruction rounds): where its result equals IEEE division and where it does
not.  These are the facts the library's arithmetic contract states
(include/jacobi.h, "Arithmetic"): the quotient is the IEEE one whenever that
is zero or a normal number; an infinite sum gives NaN; in the subnormal range
the result may be one step (2^-1074) off.

The emulation is the kernel's recipe (q0 = s * fl(1/6); r = 6 q0 - s, exact in
an FMA; q = q0 - r * fl(1/6), one FMA), written here from its definition;
Python's int / int true division rounds correctly, also into the subnormal
range, which the first test checks on ties.
"""
import math
from fractions import Fraction

import numpy as np

C = float.fromhex("0x1.5555555555555p-3")   # the double nearest 1/6
TINY = 2.0 ** -1074


def rn(v):
    """Round an exact rational to the nearest double (ties to even)."""
    return float(v)


def fma(a, b, c):
    """a * b + c with one rounding, finite operands, IEEE signed zeros."""
    v = Fraction(a) * Fraction(b) + Fraction(c)
    if v != 0:
        return rn(v)
    p_neg = (math.copysign(1.0, a) * math.copysign(1.0, b)) < 0
    c_neg = math.copysign(1.0, c) < 0
    if a * b == 0 and c == 0:
        return -0.0 if (p_neg and c_neg) else 0.0
    return 0.0   # exact cancellation of nonzero terms: +0 in round-to-nearest


def mul(a, b):
    v = Fraction(a) * Fraction(b)
    if v == 0:
        return math.copysign(0.0, a) * math.copysign(1.0, b)
    return rn(v)


def div6_three_op(s):
    q = mul(s, C)
    r = fma(6.0, q, -s)
    return fma(-r, C, q)


def same(x, y):
    return np.float64(x).view(np.uint64) == np.float64(y).view(np.uint64)


def test_rational_rounding_is_ieee_on_subnormal_ties():
    # 9 / 6 * 2^-1074 = 1.5 steps: a tie, to even (2 steps); 15 / 6 = 2.5 -> 2
    assert rn(Fraction(9, 6 * 2 ** 1074)) == 2 * TINY
    assert rn(Fraction(15, 6 * 2 ** 1074)) == 2 * TINY
    assert rn(Fraction(3, 6 * 2 ** 1074)) == 0.0


def test_normal_quotients_are_ieee():
    rng = np.random.default_rng(0)
    exps = rng.integers(-1016, 1020, 4000)
    mant = 1.0 + rng.random(4000)
    sign = np.where(rng.random(4000) < 0.5, -1.0, 1.0)
    vals = list(sign * mant * np.ldexp(1.0, exps))
    # quotients at the bottom of the normal range and sums near the top
    vals += [6 * 2.0 ** -1022, -6 * 2.0 ** -1022, np.nextafter(6 * 2.0 ** -1022, 1.0),
             np.nextafter(6 * 2.0 ** -1022, 0.0), 1.7976931348623157e308, -1.7976931348623157e308]
    vals += [float(m) for m in range(1, 600)]          # small integers, many exact quotients
    for s in vals:
        q = s / 6.0
        if q != 0 and abs(q) < 2.0 ** -1022:
            continue
        assert same(div6_three_op(s), q), s.hex()


def test_signed_zeros():
    assert same(div6_three_op(0.0), 0.0)
    assert same(div6_three_op(-0.0), -0.0)
    # tiny sums whose quotient rounds to zero keep the sign IEEE gives them
    for m in (1, 2, 3):
        assert same(div6_three_op(m * TINY), 0.0)
        assert same(div6_three_op(-m * TINY), -0.0)


def test_subnormal_quotients_off_by_at_most_one_step():
    rng = np.random.default_rng(1)
    ms = list(range(1, 2000)) + [int(x) for x in rng.integers(1, 6 * 2 ** 52, 3000)]
    off = 0
    for m in ms:
        s = m * TINY
        want = s / 6.0
        got = div6_three_op(s)
        assert abs(got - want) <= TINY, (m, got, want)
        off += got != want
        assert same(div6_three_op(-s), -got)
    # the exception is real (e.g. m = 9: a tie the three operations round down)
    assert div6_three_op(9 * TINY) == TINY and 9 * TINY / 6.0 == 2 * TINY
    assert off > 0
