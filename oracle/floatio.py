"""Multiprecision floating-point numbers and their correctly rounded matvec
(test infrastructure).

The paper's numbers are floating multiprecision values: a mantissa of b bits
(Section 2) and, in the limb form of Section 3, a per-number factor B_0 in
front of the limb sum.  Reading used here for the floating-point interface:

  * a number is a pair (M, e) of integers with |M| < 2**P, value M * 2**(e-P)
    (P significant bits; 2**(P-1) <= |M| for a normalised nonzero number, so
    the value lies in [2**(e-1), 2**e) in magnitude; M = 0 is zero);
  * the product y = A x is the exact sum, rounded once to P significant bits,
    to nearest with ties to even (the behaviour of MPFR's round-to-nearest);
    the result is normalised, and zero is (0, 0).

Storage: the significands as W = ceil((P+64)/64) little-endian two's
complement uint64 words per number (the fixed-point layout), the exponents
as a separate int32 array.
"""
from __future__ import annotations

from . import fixedpoint as fp
from . import hankel


def round_significant(S: int, E: int, P: int):
    """(M, e) of the value S * 2**E rounded to P significant bits, ties to even."""
    if S == 0:
        return 0, 0
    b = abs(S).bit_length()
    shift = b - P                      # value = (S / 2**shift) * 2**(E + shift)
    if shift <= 0:
        M = S << (-shift)
    else:
        M = fp.round_half_even(S, shift)
        if abs(M) == 1 << P:           # rounded up to the next power of two
            M >>= 1
            shift += 1
    return M, E + shift + P


def aligned_ints(Ms: list, es: list):
    """Integers N_k and a common exponent F with M_k 2**e_k = N_k 2**F exactly."""
    live = [e for M, e in zip(Ms, es) if M != 0]
    F = min(live) if live else 0
    return [M << (e - F) if M != 0 else 0 for M, e in zip(Ms, es)], F


def check_significands(Ms: list, P: int) -> None:
    lim = 1 << P
    for M in Ms:
        if not -lim < M < lim:
            raise ValueError("significand needs more than P bits")


def matvec(kind: str, Mh: list, eh: list, Mx: list, ex: list, P: int):
    """Correctly rounded y = A x for floating inputs: lists (My, ey).

    The exact sums are the schoolbook sums of eqs. (1)-(3) over the inputs
    aligned to one exponent per operand (hankel module), scaled back."""
    check_significands(Mh, P)
    check_significands(Mx, P)
    H, Fh = aligned_ints(Mh, eh)
    X, Fx = aligned_ints(Mx, ex)
    S = hankel._SUMS[kind](H, X)
    E = Fh + Fx - 2 * P                # every term is H X 2**(Fh + Fx) 2**(-2P)
    out = [round_significant(s, E, P) for s in S]
    return [m for m, _ in out], [e for _, e in out]


def decode(words, exps):
    """Significand words (count, W) and exponents -> (Ms, es) as Python ints."""
    return fp.decode(words), [int(e) for e in exps]
