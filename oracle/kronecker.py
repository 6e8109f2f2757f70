"""Whole Hankel matvec as ONE big-integer product (Kronecker substitution),
via GMP's mpz_mul through ctypes (test infrastructure).

This is a fast exact cross-check for large n: with slot width b bits, pack
A(Z) = sum_k H_k Z**k and Xr(Z) = sum_j X_{n-1-j} Z**j at Z = 2**b.  The
coefficient of Z**(i+n-1) in A * Xr is sum_j H_{i+j} X_j = S_i, the exact
Hankel sum of the schoolbook definition (Section 2, eq. (1)).  b is chosen so
every coefficient of the product lies in (-2**(b-1), 2**(b-1)), hence the
signed coefficients are recovered exactly by a balanced base-2**b read-out.
The big-integer multiply is the library primitive; packing and read-out are
plain integer bookkeeping.  Trusted only after the tests show it equals the
schoolbook sums.
"""
from __future__ import annotations

import ctypes
import ctypes.util

import numpy as np

from . import fixedpoint as fp


class _MPZ(ctypes.Structure):
    _fields_ = [("alloc", ctypes.c_int), ("size", ctypes.c_int), ("d", ctypes.c_void_p)]


_gmp = None


def _lib():
    global _gmp
    if _gmp is None:
        name = ctypes.util.find_library("gmp") or "libgmp.so.10"
        g = ctypes.CDLL(name)
        P = ctypes.POINTER(_MPZ)
        for fn, args in (("__gmpz_init", [P]), ("__gmpz_clear", [P]),
                         ("__gmpz_mul", [P, P, P]), ("__gmpz_sub", [P, P, P]),
                         ("__gmpz_mul_2exp", [P, P, ctypes.c_ulong])):
            getattr(g, fn).argtypes = args
            getattr(g, fn).restype = None
        g.__gmpz_import.argtypes = [P, ctypes.c_size_t, ctypes.c_int, ctypes.c_size_t,
                                    ctypes.c_int, ctypes.c_size_t, ctypes.c_void_p]
        g.__gmpz_import.restype = None
        g.__gmpz_export.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t),
                                    ctypes.c_int, ctypes.c_size_t, ctypes.c_int,
                                    ctypes.c_size_t, P]
        g.__gmpz_export.restype = ctypes.c_void_p
        g.__gmpz_sizeinbase.argtypes = [P, ctypes.c_int]
        g.__gmpz_sizeinbase.restype = ctypes.c_size_t
        _gmp = g
    return _gmp


def available() -> bool:
    try:
        _lib()
        return True
    except OSError:
        return False


def _signext(words: np.ndarray, Wb: int) -> np.ndarray:
    """(count, W) two's complement -> (count, Wb) sign-extended words."""
    cnt, W = words.shape
    out = np.empty((cnt, Wb), dtype=np.uint64)
    out[:, :W] = words
    neg = (words[:, W - 1] >> np.uint64(63)).astype(bool)
    out[:, W:] = np.where(neg[:, None], np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64(0))
    return out, neg


def _import_signed(g, z, words: np.ndarray, Wb: int):
    """z <- sum_k V_k 2**(64 Wb k) for the two's complement numbers V_k."""
    ext, neg = _signext(words, Wb)
    buf = np.ascontiguousarray(ext.reshape(-1))
    g.__gmpz_import(ctypes.byref(z), buf.size, -1, 8, 0, 0, buf.ctypes.data)
    # each negative V_k was read as V_k + 2**(64 Wb): subtract sum_k [V_k<0] 2**(64 Wb (k+1))
    flags = np.zeros((words.shape[0], Wb), dtype=np.uint64)
    flags[neg, 0] = 1
    fb = np.ascontiguousarray(flags.reshape(-1))
    t = _MPZ()
    g.__gmpz_init(ctypes.byref(t))
    g.__gmpz_import(ctypes.byref(t), fb.size, -1, 8, 0, 0, fb.ctypes.data)
    g.__gmpz_mul_2exp(ctypes.byref(t), ctypes.byref(t), 64 * Wb)
    g.__gmpz_sub(ctypes.byref(z), ctypes.byref(z), ctypes.byref(t))
    g.__gmpz_clear(ctypes.byref(t))


def hankel_sums(h_words, x_words, P: int) -> list:
    """Exact S_i, i = 0..n-1, from one GMP product."""
    h_words = np.ascontiguousarray(h_words, dtype=np.uint64)
    x_words = np.ascontiguousarray(x_words, dtype=np.uint64)
    n = x_words.shape[0]
    if h_words.shape[0] != 2 * n - 1:
        raise ValueError("Hankel vector must have 2n-1 entries")
    # every entry is range-checked: the slot width below assumes |X| <= 2**P
    fp.check_range(fp.decode(h_words), P)
    fp.check_range(fp.decode(x_words), P)
    # |S_i| <= n 2**(2P); slot needs 2P + log2(n) + 2 bits, rounded up to words
    Wb = max((2 * P + n.bit_length() + 2 + 63) // 64, h_words.shape[1])
    g = _lib()
    A, X, C = _MPZ(), _MPZ(), _MPZ()
    for z in (A, X, C):
        g.__gmpz_init(ctypes.byref(z))
    try:
        _import_signed(g, A, h_words, Wb)
        _import_signed(g, X, np.ascontiguousarray(x_words[::-1]), Wb)
        g.__gmpz_mul(ctypes.byref(C), ctypes.byref(A), ctypes.byref(X))
        nslots = 3 * n - 2
        nlimb = nslots * Wb + 1
        out = np.zeros(nlimb + 2, dtype=np.uint64)
        cnt = ctypes.c_size_t(0)
        g.__gmpz_export(out.ctypes.data, ctypes.byref(cnt), -1, 8, 0, 0, ctypes.byref(C))
        if cnt.value > nlimb + 2:
            raise RuntimeError("product wider than expected")
        negative = C.size < 0
    finally:
        for z in (A, X, C):
            g.__gmpz_clear(ctypes.byref(z))
    mag = int.from_bytes(out.tobytes(), "little")
    total_bits = 64 * Wb * nslots
    val = -mag if negative else mag
    u = val % (1 << total_bits)            # two's complement over all slots
    raw = u.to_bytes(total_bits // 8, "little")
    slot = 8 * Wb
    B = 1 << (64 * Wb)
    half = B >> 1
    sums = []
    carry = 0
    for t in range(2 * n - 1):             # balanced read-out, low slots first
        d = int.from_bytes(raw[t * slot:(t + 1) * slot], "little") + carry
        if d >= half:
            d -= B
            carry = 1
        else:
            carry = 0
        if t >= n - 1:
            sums.append(d)
    return sums


def hankel_matvec_words(h_words, x_words, P: int) -> np.ndarray:
    sums = hankel_sums(h_words, x_words, P)
    return fp.encode([fp.round_half_even(s, P) for s in sums], P)
