"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

This module only *draws* inputs; it holds none of the product's arithmetic.
Numbers are fixed point with P fractional bits: value = X * 2**-P with X an
integer and |X| <= 2**P.  On the wire a number is W = ceil((P + 64) / 64)
little-endian uint64 words holding X in two's complement; an array of numbers
is a C-contiguous numpy array of shape (count, W), dtype uint64.

Recipes (all deterministic from the seed tuple):

* ``uniform``: numpy ``Generator(PCG64(SeedSequence(seed)))`` draws W words per
  number, the low P+1 bits are kept as U in [0, 2**(P+1)), and X = U - 2**P,
  i.e. X is uniform on [-2**P, 2**P)  (value uniform on [-1, 1)).
* ``hilbert``: X_k = round-half-even(2**P / (k + 1)), k = 0, 1, ... (the
  Hilbert-type anti-diagonal h_k = 1/(k+1)).
* ``unit_norm``: a vector of numbers rescaled to Euclidean norm 1 (up to about
  2**-60 relative): the norm is estimated in binary64 from the leading bits,
  a 62-bit multiplier M = round(2**62 / norm) is formed, and every entry
  becomes sign(X) * floor(|X| * M / 2**62).
* ``unit``: X = 2**P at one index, zero elsewhere (a basis vector).
"""
from __future__ import annotations

import math

import numpy as np


def words_for(P: int) -> int:
    """Number of uint64 words per P-bit fixed-point number: ceil((P+64)/64)."""
    if P < 1:
        raise ValueError("P must be >= 1")
    return (P + 64 + 63) // 64


def _rng(seed) -> np.random.Generator:
    if isinstance(seed, int):
        seed = (seed,)
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(seed))))


def ints_to_words(values, P: int) -> np.ndarray:
    """Encode Python ints as (count, W) two's complement uint64 words."""
    W = words_for(P)
    buf = bytearray()
    for v in values:
        buf += int(v).to_bytes(8 * W, "little", signed=True)
    return np.frombuffer(bytes(buf), dtype="<u8").reshape(-1, W).copy()


def words_to_ints(words: np.ndarray) -> list:
    """Decode (count, W) two's complement uint64 words to Python ints."""
    words = np.ascontiguousarray(words, dtype="<u8")
    raw = words.tobytes()
    stride = 8 * words.shape[1]
    return [int.from_bytes(raw[i * stride:(i + 1) * stride], "little", signed=True)
            for i in range(words.shape[0])]


def uniform(count: int, P: int, seed) -> np.ndarray:
    """`count` numbers uniform on [-1, 1) at P fractional bits, as words."""
    W = words_for(P)
    rng = _rng(seed)
    raw = rng.integers(0, 2**64, size=(count, W), dtype=np.uint64, endpoint=False)
    # keep the low P+1 bits: U in [0, 2**(P+1))
    nb = P + 1
    full, part = divmod(nb, 64)
    if part:
        raw[:, full] &= np.uint64((1 << part) - 1)
        raw[:, full + 1:] = 0
    else:
        raw[:, full:] = 0
    # X = U - 2**P, word-wise with borrow (vectorised over numbers)
    out = raw.copy()
    wi, bi = divmod(P, 64)
    sub = np.zeros(count, dtype=np.uint64) + np.uint64(1 << bi)
    borrow = np.zeros(count, dtype=np.uint64)
    for k in range(wi, W):
        s = sub if k == wi else np.zeros(count, dtype=np.uint64)
        a = out[:, k]
        d = a - s - borrow
        borrow = ((a < s) | ((a - s) < borrow)).astype(np.uint64)
        out[:, k] = d
    return out


def hilbert(count: int, P: int) -> np.ndarray:
    """X_k = round-half-even(2**P / (k+1)) for k = 0..count-1."""
    vals = []
    one = 1 << P
    for k in range(count):
        q, r = divmod(one, k + 1)
        if 2 * r > k + 1 or (2 * r == k + 1 and (q & 1)):
            q += 1
        vals.append(q)
    return ints_to_words(vals, P)


def unit(count: int, P: int, k: int) -> np.ndarray:
    """Basis vector: X_k = 2**P, every other entry zero."""
    return ints_to_words([(1 << P) if i == k else 0 for i in range(count)], P)


def zeros(count: int, P: int) -> np.ndarray:
    return np.zeros((count, words_for(P)), dtype=np.uint64)


def unit_norm(words: np.ndarray, P: int) -> np.ndarray:
    """Rescale a vector of numbers to Euclidean norm ~1 (see module doc)."""
    vals = words_to_ints(words)
    shift = max(P - 60, 0)
    approx = [math.ldexp(float(v >> shift), shift - P) for v in vals]
    norm = math.sqrt(sum(a * a for a in approx))
    if norm == 0.0:
        return words.copy()
    M = int(round(math.ldexp(1.0, 62) / norm))
    out = []
    for v in vals:
        mag = (abs(v) * M) >> 62
        out.append(-mag if v < 0 else mag)
    return ints_to_words(out, P)


# --------------------------------------------------------------------------
# workload recipes with the paper's shapes
# --------------------------------------------------------------------------

def plain_case(n: int = 64, P: int = 3322, seed: int = 0):
    """Plain Hankel matvec: h (2n-1) and x (n) uniform on [-1, 1)."""
    return uniform(2 * n - 1, P, (1, 0, seed)), uniform(n, P, (1, 1, seed))


def hilbert_case(n: int = 1024, P: int = 33220, seed: int = 0):
    """Hilbert-type h_k = 1/(k+1) rounded to P bits; x uniform from a seed."""
    return hilbert(2 * n - 1, P), uniform(n, P, (2, 1, seed))


def session_h(n: int = 4096, P: int = 33220, seed: int = 0):
    """Resident matrix of a Lanczos-shaped session: h uniform on [-1, 1)."""
    return uniform(2 * n - 1, P, (3, 0, seed))


def session_x(n: int, P: int, k: int, seed: int = 0):
    """k-th vector of a session: uniform on [-1, 1), then unit 2-norm."""
    return unit_norm(uniform(n, P, (3, 1, seed, k)), P)


def batch_instances(count: int = 256, seed: int = 0, n_lo: int = 32, n_hi: int = 2048,
                    precisions=(1024, 4096, 16384, 33220)):
    """Uneven batch: n log-uniform in [n_lo, n_hi], P from `precisions`,
    kind = i mod 3 (0 Hankel, 1 Toeplitz, 2 circulant).  Returns a list of
    (kind, n, P) triples; the entries are drawn by `batch_operands`."""
    rng = _rng((4, 99, seed))
    out = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        P = int(precisions[int(rng.integers(0, len(precisions)))])
        out.append((i % 3, n, P))
    return out


def batch_operands(i: int, kind: int, n: int, P: int, seed: int = 0):
    hlen = n if kind == 2 else 2 * n - 1
    return uniform(hlen, P, (4, 0, seed, i)), uniform(n, P, (4, 1, seed, i))


def serving_matrices(sizes=(1000, 2000, 4000, 8000), copies: int = 2, P: int = 33220):
    """Resident matrices of the serving workload: `copies` Hankel matrices per
    n.  Returns a list of (n, P); matrix m has h = serving_h(m, n, P)."""
    return [(n, P) for _ in range(copies) for n in sizes]


def serving_h(m: int, n: int, P: int):
    return uniform(2 * n - 1, P, (5, 0, m))


def serving_x(m: int, n: int, P: int, j: int):
    """j-th vector of the pool of matrix m: uniform, then unit 2-norm."""
    return unit_norm(uniform(n, P, (5, 1, m, j)), P)


def serving_sessions(count: int, n_matrices: int, seed: int = 0, len_lo: int = 50,
                     len_hi: int = 300):
    """Session descriptors (matrix index, number of matvecs), drawn uniformly."""
    rng = _rng((5, 2, seed))
    return [(int(rng.integers(0, n_matrices)), int(rng.integers(len_lo, len_hi + 1)))
            for _ in range(count)]
