"""Fixed-point number format and the one rounding step (test infrastructure).

A number is X * 2**-P with X an integer; inputs satisfy |X| <= 2**P.  It is
stored as W = ceil((P+64)/64) little-endian uint64 words, two's complement.

The paper computes with floating multiprecision numbers (mantissa of b bits,
Section 2 and the limb form of Section 3) and never fixes a rounding rule.
Reading used here: fixed point with P fractional bits, the exact integer
result is rounded once, to nearest with ties to even, at 2**-P.
"""
from __future__ import annotations

import numpy as np


def words_for(P: int) -> int:
    return (P + 127) // 64


def decode(words) -> list:
    """(count, W) uint64 two's complement words -> list of Python ints."""
    a = np.ascontiguousarray(words, dtype="<u8")
    if a.ndim != 2:
        raise ValueError("expected a (count, W) array")
    raw = a.tobytes()
    s = 8 * a.shape[1]
    return [int.from_bytes(raw[i * s:(i + 1) * s], "little", signed=True)
            for i in range(a.shape[0])]


def encode(values, P: int) -> np.ndarray:
    """Python ints -> (count, W) uint64 words; raises if a value does not fit."""
    W = words_for(P)
    out = bytearray()
    for v in values:
        out += int(v).to_bytes(8 * W, "little", signed=True)   # OverflowError if too wide
    return np.frombuffer(bytes(out), dtype="<u8").reshape(-1, W).copy()


def check_range(values, P: int) -> None:
    """Inputs must satisfy |X| <= 2**P (value in [-1, 1])."""
    lim = 1 << P
    for v in values:
        if v > lim or v < -lim:
            raise ValueError("input magnitude exceeds 1")


def round_half_even(S: int, P: int) -> int:
    """Nearest integer to S / 2**P, ties to the even neighbour."""
    q, r = divmod(S, 1 << P)          # floor division: 0 <= r < 2**P
    half = 1 << (P - 1)
    if r > half or (r == half and (q & 1)):
        q += 1
    return q
