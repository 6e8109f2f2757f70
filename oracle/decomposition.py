"""Section 3 (the decomposition approach), in exact integers (test
infrastructure, small cases only).

The paper writes every multiprecision number as a sum of limbs
a = B_0 * sum_k B**k a_k and recovers y from a product of the limb terms
(eq. (5) sums blocks of the auxiliary product).  The exact analogue used as a
pin: keep the limb weight as a formal variable z = 2**w, so each number is a
polynomial with small integer coefficients, form the bivariate
index-by-limb correlation S_i(z) = sum_j H_i+j(z) X_j(z) exactly, and evaluate
at z = 2**w.  The limbs here are balanced base-2**w digits in
[-2**(w-1), 2**(w-1)).
"""
from __future__ import annotations


def balanced_digits(X: int, w: int, L: int) -> list:
    """Digits d_0..d_{L-1} in [-2**(w-1), 2**(w-1)) with X = sum d_e 2**(w e).
    Raises if X does not fit in L balanced digits."""
    B = 1 << w
    half = B >> 1
    out = []
    v = X
    for _ in range(L):
        d = v % B                      # 0 <= d < B
        if d >= half:
            d -= B
        out.append(d)
        v = (v - d) >> w               # exact
    if v != 0:
        raise ValueError("value does not fit in L balanced digits")
    return out


def poly_mul(a: list, b: list) -> list:
    out = [0] * (len(a) + len(b) - 1)
    for i, ai in enumerate(a):
        if ai:
            for j, bj in enumerate(b):
                out[i + j] += ai * bj
    return out


def hankel_limb_coeffs(H: list, X: list, w: int, L: int) -> list:
    """Exact limb coefficients s_{i,e} of S_i(z) = sum_j H_{i+j}(z) X_j(z)."""
    n = len(X)
    Hd = [balanced_digits(v, w, L) for v in H]
    Xd = [balanced_digits(v, w, L) for v in X]
    rows = []
    for i in range(n):
        acc = [0] * (2 * L - 1)
        for j in range(n):
            for e, c in enumerate(poly_mul(Hd[i + j], Xd[j])):
                acc[e] += c
        rows.append(acc)
    return rows


def evaluate(coeffs: list, w: int) -> int:
    """sum_e s_e 2**(w e)."""
    return sum(c << (w * e) for e, c in enumerate(coeffs))
