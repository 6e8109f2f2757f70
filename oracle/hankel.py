"""Schoolbook structured matvecs in exact integers (test infrastructure).

Definitions followed (paper, Section 2 "Preliminaries"):
  * Hankel, eq. (1): A_H[i][j] = a_{i+j-1} (1-based), the matrix is given by
    the vector a_1..a_{2n-1}.  0-based here: A[i][j] = h[i+j].
  * Toeplitz, eq. (2): A_T[i][j] = a_{n-i+j}, same vector a.  0-based:
    A[i][j] = h[n-1-i+j], i.e. the Hankel matrix with its rows reversed.
  * Circulant, eq. (3): first column a_1..a_n, A_C[i][j] = a_{((i-j) mod n)+1}.
    0-based: A[i][j] = c[(i-j) mod n], c of length n.
  * The schoolbook product (the sum printed right after eq. (3)); its
    summation index is garbled in print, the reading is
    y_i = sum_j a_{i+j-1} x_j, the row of eq. (1) times x.

Each entry of y is the exact integer sum rounded once (fixedpoint module).
"""
from __future__ import annotations

from . import fixedpoint as fp


def hankel_sums(H: list, X: list) -> list:
    """Exact S_i = sum_j H[i+j] * X[j], i = 0..n-1 (len(H) = 2n-1)."""
    n = len(X)
    if len(H) != 2 * n - 1:
        raise ValueError("Hankel vector must have 2n-1 entries")
    return [sum(H[i + j] * X[j] for j in range(n)) for i in range(n)]


def toeplitz_sums(H: list, X: list) -> list:
    """Exact S_i = sum_j H[n-1-i+j] * X[j] (eq. (2), 0-based)."""
    n = len(X)
    if len(H) != 2 * n - 1:
        raise ValueError("Toeplitz vector must have 2n-1 entries")
    return [sum(H[n - 1 - i + j] * X[j] for j in range(n)) for i in range(n)]


def circulant_sums(C: list, X: list) -> list:
    """Exact S_i = sum_j C[(i-j) mod n] * X[j] (eq. (3), 0-based)."""
    n = len(X)
    if len(C) != n:
        raise ValueError("circulant vector must have n entries")
    return [sum(C[(i - j) % n] * X[j] for j in range(n)) for i in range(n)]


_SUMS = {"hankel": hankel_sums, "toeplitz": toeplitz_sums, "circulant": circulant_sums}


def matvec_ints(kind: str, H: list, X: list, P: int) -> list:
    """Correctly rounded y (as integers Y_i, value Y_i * 2**-P)."""
    fp.check_range(H, P)
    fp.check_range(X, P)
    return [fp.round_half_even(s, P) for s in _SUMS[kind](H, X)]


def matvec_words(kind: str, h_words, x_words, P: int):
    """Word-level oracle: decode, exact product, round, encode."""
    H = fp.decode(h_words)
    X = fp.decode(x_words)
    return fp.encode(matvec_ints(kind, H, X, P), P)


def hankel_row(H: list, X: list, i: int) -> int:
    """One exact Hankel sum S_i (for sampled checks at large n)."""
    return sum(H[i + j] * X[j] for j in range(len(X)))


_SHARED = None   # (kind, H, X, P) inherited by forked workers


def _row_value(kind, H, X, i, P):
    n = len(X)
    if kind == "hankel":
        s = sum(H[i + j] * X[j] for j in range(n))
    elif kind == "toeplitz":
        s = sum(H[n - 1 - i + j] * X[j] for j in range(n))
    else:
        s = sum(H[(i - j) % n] * X[j] for j in range(n))
    return fp.round_half_even(s, P)


def _row_worker(i):
    kind, H, X, P = _SHARED
    return _row_value(kind, H, X, i, P)


def matvec_rows(kind: str, H: list, X: list, P: int, rows, processes: int = 1) -> list:
    """Correctly rounded Y_i for the given rows only, optionally over a
    fork-based process pool (the operands are inherited, not pickled)."""
    global _SHARED
    fp.check_range(H, P)
    fp.check_range(X, P)
    rows = [int(i) for i in rows]
    if processes <= 1 or len(rows) <= 1:
        return [_row_value(kind, H, X, i, P) for i in rows]
    import multiprocessing as mp
    _SHARED = (kind, H, X, P)
    try:
        with mp.get_context("fork").Pool(processes) as pool:
            return pool.map(_row_worker, rows, chunksize=1)
    finally:
        _SHARED = None
