"""Section 4, Algorithm 1: the recursive half-size Hankel product, in exact
integers (test infrastructure).

Notation follows the paper: the matrix is the vector a_1..a_{2n-1}, the input
x_1..x_n, the output y_1..y_n (1-based; a list slot 0 is unused).  One level
builds, with m = floor((n+1)/2) and m1 = ceil((n+1)/2),
  h_i = x_{2i-1},  f_i = x_{2i-1} - x_{2i}             (i = 1..m)
  c_i = a_{2i-1} + a_{2i},  d_i = a_{2i}               (i = 1..2m-1)
  g_i = x_{2i-2} - x_{2i-1}                            (i = 1..m1)
  e_i = a_{2i-1}                                       (i = 1..2m1-1)
with x_0 = x_{n+1} = 0 and a_{2n} = a_{2n+1} = 0, recurses on
p = C h, q = D f (size m) and r = E g (size m1), and combines
  y_{2i-1} = p_i - q_i,   y_{2i} = p_i + r_i  (when 2i <= n).

Readings (the paper only gives the n = 2 base case; a call with n = 1 would
recurse on itself since then m = m1 = 1):
  * base case n = 1: y_1 = a_1 x_1;
  * optional schoolbook cutoff n0: sizes n <= n0 use the plain sum; the
    result is the same exact integer vector.
The step list is authoritative over the prose before it where the two differ
in index ranges (the prose gives d over m entries; the step list over 2m-1).
"""
from __future__ import annotations


def _pad(v):
    return [None] + list(v)


def alg1(n: int, a: list, x: list, n0: int = 2) -> list:
    """Exact y = A_H x by Algorithm 1.  a has 2n-1 entries, x has n (0-based
    Python lists in, 0-based list out)."""
    if len(a) != 2 * n - 1 or len(x) != n:
        raise ValueError("shape mismatch")
    return _alg1(n, _pad(a), _pad(x), max(n0, 2))[1:]


def _get(v, k, hi):
    """v_k with the zero conventions outside 1..hi."""
    return v[k] if 1 <= k <= hi else 0


def _alg1(n, a, x, n0):
    if n == 1:
        return [None, a[1] * x[1]]
    if n == 2:
        return [None, a[1] * x[1] + a[2] * x[2], a[2] * x[1] + a[3] * x[2]]
    if n <= n0:
        return [None] + [sum(a[i + j - 1] * x[j] for j in range(1, n + 1))
                         for i in range(1, n + 1)]
    m = (n + 1) // 2
    m1 = (n + 2) // 2
    A = 2 * n - 1
    h = [None] * (m + 1)
    f = [None] * (m + 1)
    for i in range(1, m + 1):
        f[i] = _get(x, 2 * i - 1, n) - _get(x, 2 * i, n)
        h[i] = _get(x, 2 * i - 1, n)
    c = [None] * (2 * m)
    d = [None] * (2 * m)
    for i in range(1, 2 * m):
        c[i] = _get(a, 2 * i - 1, A) + _get(a, 2 * i, A)
        d[i] = _get(a, 2 * i, A)
    g = [None] * (m1 + 1)
    for i in range(1, m1 + 1):
        g[i] = _get(x, 2 * i - 2, n) - _get(x, 2 * i - 1, n)
    e = [None] * (2 * m1)
    for i in range(1, 2 * m1):
        e[i] = _get(a, 2 * i - 1, A)
    p = _alg1(m, c, h, n0)
    q = _alg1(m, d, f, n0)
    r = _alg1(m1, e, g, n0)
    y = [None] * (n + 1)
    for i in range(1, m + 1):
        y[2 * i - 1] = p[i] - q[i]
        if 2 * i <= n:
            y[2 * i] = p[i] + r[i]
    return y


def mult_count(n: int, n0: int = 2) -> int:
    """Scalar multiplications Algorithm 1 performs as implemented above:
    M(1) = 1, M(2) = 4, M(n) = n*n for n <= n0, else
    M(n) = 2 M(floor((n+1)/2)) + M(ceil((n+1)/2))."""
    memo = {}

    def M(k):
        if k in memo:
            return memo[k]
        if k == 1:
            v = 1
        elif k == 2:
            v = 4
        elif k <= max(n0, 2):
            v = k * k
        else:
            v = 2 * M((k + 1) // 2) + M((k + 2) // 2)
        memo[k] = v
        return v

    return M(n)
