"""Pins of the floating-point oracle (oracle/floatio.py) against exact
rationals, hand-derived roundings and invariants (CPU only)."""
import random
from fractions import Fraction

import pytest

from oracle import floatio, hankel


def _value(M, e, P):
    return Fraction(M) * Fraction(2) ** (e - P)


def _round_fraction(v: Fraction, P: int):
    """Independent rounding of an exact rational to P significant bits, ties
    to even, by comparison with powers of two (no integer shifting)."""
    if v == 0:
        return 0, 0
    a = abs(v)
    e = 0
    while a >= Fraction(2) ** e:
        e += 1
    while a < Fraction(2) ** (e - 1):
        e -= 1
    # 2**(e-1) <= a < 2**e: the significand is a * 2**(P-e) in [2**(P-1), 2**P)
    t = v * Fraction(2) ** (P - e)
    fl = t.numerator // t.denominator
    frac = t - fl
    if frac > Fraction(1, 2) or (frac == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    if abs(fl) == 2 ** P:
        fl //= 2
        e += 1
    return fl, e


def _brute(kind, Mh, eh, Mx, ex, P):
    n = len(Mx)
    hv = [_value(m, e, P) for m, e in zip(Mh, eh)]
    xv = [_value(m, e, P) for m, e in zip(Mx, ex)]
    rows = []
    for i in range(n):
        s = Fraction(0)
        for j in range(n):
            if kind == "hankel":
                a = hv[i + j]
            elif kind == "toeplitz":
                a = hv[n - 1 - i + j]
            else:
                a = hv[(i - j) % n]
            s += a * xv[j]
        rows.append(_round_fraction(s, P))
    return [m for m, _ in rows], [e for _, e in rows]


def _rand_float(rng, P, elo, ehi):
    M = rng.randrange(-(2 ** P) + 1, 2 ** P)
    return M, rng.randrange(elo, ehi)


@pytest.mark.parametrize("kind", ["hankel", "toeplitz", "circulant"])
def test_equals_exact_rationals(kind):
    rng = random.Random(11)
    for _ in range(60):
        n = rng.randrange(1, 7)
        P = rng.choice([1, 2, 3, 5, 8, 13, 64, 65, 100])
        spread = rng.choice([0, 3, 40, 300])
        hl = n if kind == "circulant" else 2 * n - 1
        h = [_rand_float(rng, P, -spread - 5, spread + 5) for _ in range(hl)]
        x = [_rand_float(rng, P, -spread - 5, spread + 5) for _ in range(n)]
        if rng.random() < 0.3:
            h[rng.randrange(hl)] = (0, 0)
        Mh, eh = [m for m, _ in h], [e for _, e in h]
        Mx, ex = [m for m, _ in x], [e for _, e in x]
        got = floatio.matvec(kind, Mh, eh, Mx, ex, P)
        assert got == _brute(kind, Mh, eh, Mx, ex, P), (kind, n, P, spread)


def test_round_significant_hand_cases():
    # 23 = 10111b to 4 bits: a tie between 1011 and 1100 -> even 1100 (12);
    # the value 23 * 2**E becomes 12 * 2**(E+1), so e = E + 1 + 4
    assert floatio.round_significant(23, 0, 4) == (12, 5)
    # 21 = 10101b: 1010|1 is a tie, 1010 is even -> 10 * 2**1
    assert floatio.round_significant(21, 0, 4) == (10, 5)
    assert floatio.round_significant(-23, 0, 4) == (-12, 5)
    # 31 = 11111b: rounds up to 10000|0 -> renormalised to 8 * 2**2
    assert floatio.round_significant(31, -3, 4) == (8, -3 + 2 + 4)
    # already short: scaled up, exact
    assert floatio.round_significant(3, 7, 4) == (12, 7 - 2 + 4)
    # 81 / 256 = 1010001b * 2**-8 -> 1010 * 2**-5 = 10 * 2**(e-4) with e = -1
    assert floatio.round_significant(81, -8, 4) == (10, -1)
    assert floatio.round_significant(0, 99, 4) == (0, 0)


def test_product_of_two_nines():
    # n = 1, P = 4: (9/16) * (9/16) = 81/256 -> 10 * 2**(-1-4)
    assert floatio.matvec("hankel", [9], [0], [9], [0], 4) == ([10], [-1])


def test_tie_through_a_sum():
    # y_0 = 4 * 4 * 2**-8 + 7 * 1 * 2**-8 = 23 * 2**-8 -> tie -> 12 * 2**(-7-4)
    P = 4
    Mh, eh = [4, 7, 0], [0, 0, 0]
    Mx, ex = [4, 1], [0, 0]
    My, ey = floatio.matvec("hankel", Mh, eh, Mx, ex, P)
    assert (My[0], ey[0]) == (12, -3)
    assert _value(12, -3, P) == Fraction(24, 256)


def test_exact_cancellation_is_zero():
    P = 10
    # y_0 = a x0 + b x1 with b x1 = -a x0 at different exponents
    Mh, eh = [3, -6, 0], [5, 4, 0]
    Mx, ex = [5, 5], [2, 2]
    My, ey = floatio.matvec("hankel", Mh, eh, Mx, ex, P)
    assert (My[0], ey[0]) == (0, 0)


def test_exponent_shift_invariance():
    rng = random.Random(12)
    for _ in range(30):
        n, P = rng.randrange(1, 6), rng.choice([7, 33, 64])
        h = [_rand_float(rng, P, -50, 50) for _ in range(2 * n - 1)]
        x = [_rand_float(rng, P, -50, 50) for _ in range(n)]
        k = rng.randrange(-1000, 1000)
        Mh, eh = [m for m, _ in h], [e for _, e in h]
        Mx, ex = [m for m, _ in x], [e for _, e in x]
        My, ey = floatio.matvec("hankel", Mh, eh, Mx, ex, P)
        My2, ey2 = floatio.matvec("hankel", Mh, [e + k for e in eh], Mx, ex, P)
        assert My2 == My
        assert ey2 == [e + k if m != 0 else 0 for e, m in zip(ey, My)]


def test_equal_exponents_reduce_to_the_fixed_point_sums():
    rng = random.Random(13)
    P, n = 50, 5
    H = [rng.randrange(-(2 ** P) + 1, 2 ** P) for _ in range(2 * n - 1)]
    X = [rng.randrange(-(2 ** P) + 1, 2 ** P) for _ in range(n)]
    My, ey = floatio.matvec("hankel", H, [0] * len(H), X, [0] * n, P)
    for S, m, e in zip(hankel.hankel_sums(H, X), My, ey):
        # value = S 2**-2P: m 2**(e-P) is its P-bit rounding, within half an ulp
        err = abs(Fraction(S, 2 ** (2 * P)) - _value(m, e, P))
        assert err <= Fraction(2) ** (e - P - 1)
        assert 2 ** (P - 1) <= abs(m) < 2 ** P


def test_significand_range_is_checked():
    with pytest.raises(ValueError):
        floatio.matvec("hankel", [16], [0], [1], [0], 4)
