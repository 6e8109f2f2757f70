"""Section 4, Algorithm 1: the recursive half-size Hankel product, in exact
integers (test infrastructure).

What one level of the recursion rests on.  Write the Hankel product as
y_i = sum_j a_{i+j} x_j (0-based here: a has 2n-1 entries, x and y have n)
and pair the rows and the columns two by two.  With x padded by zeros
(x_{-1} = x_n = 0) and a padded by zeros past its end, the even and odd
output rows are

    y_{2i}   = p_i - q_i,        y_{2i+1} = p_i + r_i,

where p, q and r are Hankel products of about half the size:

    p = C u,  C_t = a_{2t} + a_{2t+1},  u_k = x_{2k}             (m entries)
    q = D f,  D_t = a_{2t+1},           f_k = x_{2k} - x_{2k+1}  (m entries)
    r = E g,  E_t = a_{2t},             g_k = x_{2k-1} - x_{2k}  (m1 entries)

with m = floor((n+1)/2) and m1 = ceil((n+1)/2) (C and D have 2m-1 entries,
E has 2m1-1).  This is the paper's identity y = Ch - Df on odd rows and
y = Ch + Eg on even ones (1-based rows), three products of half size in
place of four.  Each of p, q, r is computed by the same recursion.

Readings (the paper gives only the n = 2 base case, and a call with n = 1
would recurse on itself since then m = m1 = 1):
  * sizes n <= n0 (n0 >= 2) use the plain sum; for n = 1 and n = 2 that is
    the paper's base case, and a larger n0 gives the same exact result;
  * where the paper's prose and its step list give different index ranges
    for the auxiliary vectors, the step list is followed (D over 2m-1
    entries, E over 2m1-1).
"""
from __future__ import annotations


def _plain(a: list, x: list) -> list:
    n = len(x)
    return [sum(a[i + j] * x[j] for j in range(n)) for i in range(n)]


def _padded(v: list, length: int, lead: int = 0) -> list:
    """`lead` zeros, then v, then zeros up to `length` entries in all."""
    out = [0] * lead + list(v)
    return out + [0] * (length - len(out))


def _half_products(a: list, x: list, n0: int) -> list:
    n = len(x)
    if n <= n0:
        return _plain(a, x)
    m = (n + 1) // 2
    m1 = (n + 2) // 2
    xs = _padded(x, 2 * m)                  # x_0 .. x_{2m-1}, zero past x_{n-1}
    xg = _padded(x, 2 * m1, lead=1)         # x_{-1} .. x_{2m1-2}
    ap = _padded(a, 2 * (2 * m1 - 1))       # a past a_{2n-2} is zero
    u = xs[0::2]
    f = [e - o for e, o in zip(xs[0::2], xs[1::2])]
    g = [e - o for e, o in zip(xg[0::2], xg[1::2])]
    C = [ap[2 * t] + ap[2 * t + 1] for t in range(2 * m - 1)]
    D = ap[1:2 * (2 * m - 1):2]
    E = ap[0:2 * (2 * m1 - 1):2]
    p = _half_products(C, u, n0)
    q = _half_products(D, f, n0)
    r = _half_products(E, g, n0)
    y = [0] * n
    y[0::2] = [pi - qi for pi, qi in zip(p, q)]                  # m even rows
    y[1::2] = [pi + ri for pi, ri in zip(p, r)][:n // 2]         # n//2 odd rows
    return y


def alg1(n: int, a: list, x: list, n0: int = 2) -> list:
    """Exact y = A_H x by the recursion above.  a has 2n-1 entries, x has n
    (0-based Python lists in, 0-based list out)."""
    if len(a) != 2 * n - 1 or len(x) != n:
        raise ValueError("shape mismatch")
    return _half_products(list(a), list(x), max(n0, 2))


def mult_count(n: int, n0: int = 2) -> int:
    """Scalar multiplications the recursion performs: M(n) = n*n for
    n <= max(n0, 2), else M(n) = 2 M(floor((n+1)/2)) + M(ceil((n+1)/2))."""
    memo = {}

    def M(k):
        if k not in memo:
            if k <= max(n0, 2):
                memo[k] = k * k
            else:
                memo[k] = 2 * M((k + 1) // 2) + M((k + 2) // 2)
        return memo[k]

    return M(n)
